// 3D U-Net surrogate (paper Sec. 4, Table 2; architecture of App. A.2) on
// gfx950 behind the C ABI of include/mi355lbm.h: forward pass, masked-MSE
// backward pass and Adam, with the kernels of unet_kernels.h.
//
// Network: encoder stages of widths w0..w3, each two blocks of 3x3x3
// convolution, batch normalisation and ReLU, then 2x2x2 max pooling; a
// bottleneck of two blocks; a decoder that upsamples trilinearly by two,
// concatenates the skip connection of the same level (upsampled channels
// first) and applies two blocks; a 1x1x1 convolution with bias and a
// sigmoid.  Convolutions have no bias and pad by one cell.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mi355lbm.h"
#include "unet_kernels.h"

using namespace munet;

namespace {

struct Blk {
  int cin, cind, cout;  // input channels (parameters, device), output channels
  int level;            // spatial level (0 = full resolution, 4 = bottleneck)
  int64_t woff, goff, boff;       // offsets of W [cout][cin][27], gamma, beta
  uint16_t* wt = nullptr; int kp = 0, coutp = 0;   // forward operand [coutp][kp]
  uint16_t* wb = nullptr; int kpb = 0, rowsb = 0;  // adjoint operand [rowsb][kpb]
  float* z = nullptr;      // conv output FP32 [V][cout]
  uint16_t* a = nullptr;   // activation BF16 [V][cout]
  float* g = nullptr;      // dL/da FP32 [V][cout]
  uint16_t* dz = nullptr;  // dL/dz BF16 [V][cout]
  float *mean = nullptr, *istd = nullptr, *scale = nullptr, *shift = nullptr, *rmean = nullptr, *rvar = nullptr,
        *coef = nullptr;
  int64_t rs_off = 0;      // offset of its channels in the running-statistics vectors
};

}  // namespace

struct unet_net {
  unet_params p{};
  hipStream_t st = nullptr;
  int dims[5][3];
  std::vector<Blk> blk;     // enc0a enc0b ... enc3b bota botb dec3a dec3b ... dec0a dec0b
  int64_t nparam = 0, head_w = 0, head_b = 0, nbn = 0;
  float *theta = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
  uint16_t* xin = nullptr;
  uint16_t* pool[4] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t* up[4] = {nullptr, nullptr, nullptr, nullptr};
  float* gpool[4] = {nullptr, nullptr, nullptr, nullptr};
  float* gcat[4] = {nullptr, nullptr, nullptr, nullptr};
  float* stats = nullptr;   // conv statistics / BN adjoint partials
  float* part = nullptr;    // weight-gradient partials
  int64_t part_cap = 0;
  float* hpart = nullptr;
  uint16_t* dlog = nullptr;
  float* y = nullptr;       // forward output of the last training pass [B][cout][P]
  double* dscal = nullptr;  // [0] mask count, [1] loss
  int64_t adam_t = 0;
  std::vector<void*> allocs;
  std::string err;
};

static std::string g_unet_err;

static int ufail(unet_net* n, int code, const std::string& m) {
  if (n) n->err = m;
  g_unet_err = m;
  return code;
}

#define UCHK(n, call)                                                                                          \
  do {                                                                                                         \
    hipError_t e_ = (call);                                                                                    \
    if (e_ != hipSuccess)                                                                                      \
      return ufail((n), e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,                                  \
                   std::string(#call) + ": " + hipGetErrorString(e_));                                         \
  } while (0)

static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }
static inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

static bool pow2_width(int c) { return c >= 8 && c <= 2048 && (c & (c - 1)) == 0; }

static int check_params(const unet_params& p) {
  if (p.nx <= 0 || p.ny <= 0 || p.nz <= 0 || p.nx % 16 || p.ny % 16 || p.nz % 16)
    return ufail(nullptr, LBM_EINVAL, "grid must be positive multiples of 16 (four poolings)");
  if (p.cin < 1 || p.cin > 8 || p.cout < 1 || p.cout > 8) return ufail(nullptr, LBM_EINVAL, "cin, cout must be 1..8");
  for (int l = 0; l < 4; ++l)
    if (!pow2_width(p.widths[l])) return ufail(nullptr, LBM_EINVAL, "widths must be powers of two in [8, 2048]");
  if (!pow2_width(p.bottleneck)) return ufail(nullptr, LBM_EINVAL, "bottleneck must be a power of two in [8, 2048]");
  if (p.max_batch < 1) return ufail(nullptr, LBM_EINVAL, "max_batch must be positive");
  return LBM_OK;
}

// block table in forward order, with parameter offsets
static void build_blocks(const unet_params& p, std::vector<Blk>& b, int64_t& nparam, int64_t& hw, int64_t& hb,
                         int64_t& nbn) {
  b.clear();
  int64_t off = 0, rs = 0;
  auto add = [&](int cin, int cout, int level) {
    Blk k;
    k.cin = cin;
    k.cind = cin < 8 ? 8 : cin;
    k.cout = cout;
    k.level = level;
    k.woff = off;
    off += (int64_t)cout * cin * 27;
    k.goff = off;
    off += cout;
    k.boff = off;
    off += cout;
    k.rs_off = rs;
    rs += cout;
    b.push_back(k);
  };
  int c = p.cin;
  for (int l = 0; l < 4; ++l) {
    add(c, p.widths[l], l);
    add(p.widths[l], p.widths[l], l);
    c = p.widths[l];
  }
  add(c, p.bottleneck, 4);
  add(p.bottleneck, p.bottleneck, 4);
  c = p.bottleneck;
  for (int l = 3; l >= 0; --l) {
    add(c + p.widths[l], p.widths[l], l);
    add(p.widths[l], p.widths[l], l);
    c = p.widths[l];
  }
  hw = off;
  off += (int64_t)p.cout * p.widths[0];
  hb = off;
  off += p.cout;
  nparam = off;
  nbn = rs;
}

// indices in the block table
static inline int ienc(int l, int h) { return 2 * l + h; }
static inline int ibot(int h) { return 8 + h; }
static inline int idec(int l, int h) { return 10 + 2 * (3 - l) + h; }

extern "C" int64_t unet_param_count(const unet_params* p) {
  if (!p || check_params(*p)) return -1;
  std::vector<Blk> b;
  int64_t n, hw, hb, nbn;
  build_blocks(*p, b, n, hw, hb, nbn);
  return n;
}

static void free_unet(unet_net* n) {
  for (void* q : n->allocs) (void)hipFree(q);
  n->allocs.clear();
}

template <typename T>
static int ualloc(unet_net* n, T** ptr, size_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes < 256 ? 256 : bytes);
  if (e != hipSuccess) return ufail(n, e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "device allocation failed");
  n->allocs.push_back(q);
  *ptr = (T*)q;
  return LBM_OK;
}

static int64_t vox(const unet_net* n, int level, int B) {
  return (int64_t)B * n->dims[level][0] * n->dims[level][1] * n->dims[level][2];
}

// chunking of the LDS weight-gradient kernel: about 1024 blocks over the
// (chunk, 32 output channels, citiles input-channel tiles) grid
static int wgrad_lds_chunks(int64_t nbox, int cout, int citiles, int64_t& per_chunk) {
  const int64_t tiles = (int64_t)(cout / 32) * citiles;
  int64_t nc = std::max<int64_t>(1, (1024 + tiles - 1) / tiles);
  nc = std::min<int64_t>(nc, nbox);
  per_chunk = (nbox + nc - 1) / nc;
  return (int)((nbox + per_chunk - 1) / per_chunk);
}

// tiling of the LDS weight gradient for inputs of c0 + c1 channels on a
// grid d: the box depth (16 or 8; 0 where the kernel does not apply) and
// the input-channel tile ci (32, or 8 for the 8-channel input layer, which
// has an instance for 16-deep boxes only)
static int lds_tiling(int c0, int c1, const int* d, int& ci) {
  ci = c0 % 32 == 0 && c1 % 32 == 0 ? 32 : (c0 == 8 && c1 == 0 ? 8 : 0);
  if (!ci || d[0] % CL_TX || d[1] % WL_TY) return 0;
  const int tz = d[2] % 16 == 0 ? 16 : (d[2] % 8 == 0 ? 8 : 0);
  return ci == 8 && tz != 16 ? 0 : tz;
}

// chunking of a weight-gradient reduction over V voxels for a (cout, K) tile grid
static void wgrad_chunks(int64_t V, int cout, int K, int& nchunk, int64_t& chunk) {
  const int tiles = ((cout + 63) / 64) * ((K + 63) / 64);
  const int64_t steps = (V + 63) / 64;
  int64_t nc = std::max<int64_t>(1, 2048 / tiles);
  nc = std::min<int64_t>(nc, steps);
  chunk = 64 * ((steps + nc - 1) / nc);
  nchunk = (int)((V + chunk - 1) / chunk);
}

// k splits of the direct convolution over V voxels with rows output rows
// and kp k: a grid of fewer than 512 blocks (the bottleneck) is split over
// k towards 1024 blocks, at least 16 k steps of 32 per split
static int conv_splits(int64_t V, int rows, int kp) {
  const int64_t blocks = ((V + CV_VOX - 1) / CV_VOX) * (rows / CV_CO);
  if (blocks >= 512) return 1;
  const int64_t ks = std::min<int64_t>((1024 + blocks - 1) / blocks, (kp / 32) / 16);
  return (int)std::max<int64_t>(ks, 1);
}

// re-derive the BF16 operands of every convolution from the FP32 parameters
static int repack(unet_net* n) {
  for (auto& k : n->blk) {
    hipLaunchKernelGGL(pack_fwd_kernel, dim3(nb256((int64_t)k.coutp * k.kp)), dim3(256), 0, n->st,
                       n->theta + k.woff, k.cout, k.cin, k.cind, 27, k.coutp, k.kp, k.wt);
    hipLaunchKernelGGL(pack_bwd_kernel, dim3(nb256((int64_t)k.rowsb * k.kpb)), dim3(256), 0, n->st,
                       n->theta + k.woff, k.cout, k.cin, 27, k.rowsb, k.kpb, k.wb);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ufail(n, LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

extern "C" int unet_create(const unet_params* pin, uint64_t seed, void* hip_stream, unet_net** out) {
  if (!pin || !out) return ufail(nullptr, LBM_EINVAL, "null argument");
  *out = nullptr;
  if (int rc = check_params(*pin)) return rc;
  unet_net* n = new (std::nothrow) unet_net();
  if (!n) return ufail(nullptr, LBM_ENOMEM, "host allocation failed");
  n->p = *pin;
  n->st = (hipStream_t)hip_stream;
  for (int l = 0; l < 5; ++l) {
    n->dims[l][0] = pin->nx >> l;
    n->dims[l][1] = pin->ny >> l;
    n->dims[l][2] = pin->nz >> l;
  }
  build_blocks(*pin, n->blk, n->nparam, n->head_w, n->head_b, n->nbn);
  const int B = pin->max_batch;
  auto bail = [&](int rc) {
    free_unet(n);
    delete n;
    return rc;
  };
#define UA(ptr, bytes) \
  if (int rc_ = ualloc(n, &(ptr), (size_t)(bytes))) return bail(rc_)
  UA(n->theta, n->nparam * 4);
  UA(n->grad, n->nparam * 4);
  UA(n->am, n->nparam * 4);
  UA(n->av, n->nparam * 4);
  float* rsbuf = nullptr;
  UA(rsbuf, n->nbn * 4 * 2);
  int64_t stats_cap = 0;
  n->part_cap = 0;
  for (auto& k : n->blk) {
    const int64_t V = vox(n, k.level, B);
    k.kp = round_up(27 * k.cind, 32);
    k.coutp = round_up(k.cout, CV_CO);
    k.kpb = round_up(27 * k.cout, 32);
    k.rowsb = round_up(k.cind, CV_CO);
    UA(k.wt, (int64_t)k.coutp * k.kp * 2);
    UA(k.wb, (int64_t)k.rowsb * k.kpb * 2);
    UA(k.z, V * k.cout * 4);
    UA(k.a, V * k.cout * 2);
    UA(k.g, V * k.cout * 4);
    UA(k.dz, V * k.cout * 2);
    UA(k.mean, k.cout * 4);
    UA(k.istd, k.cout * 4);
    UA(k.scale, k.cout * 4);
    UA(k.shift, k.cout * 4);
    UA(k.coef, k.cout * 12);
    k.rmean = rsbuf + k.rs_off;
    k.rvar = rsbuf + n->nbn + k.rs_off;
    stats_cap = std::max<int64_t>(stats_cap, (int64_t)nb256(V) * k.cout * 2);
    // statistics per CSR_VOX voxels after a k split (at any batch: one
    // sample has the fewest blocks)
    if (conv_splits(V / B, k.coutp, k.kp) > 1)
      stats_cap = std::max<int64_t>(stats_cap, (V + CSR_VOX - 1) / CSR_VOX * k.cout * 2);
    int nc;
    int64_t ch;
    wgrad_chunks(V, k.cout, 27 * k.cind, nc, ch);
    n->part_cap = std::max<int64_t>(n->part_cap, (int64_t)nc * k.cout * 27 * k.cind);
    int ci = 0;
    if (const int tz = k.cout % 32 == 0 ? lds_tiling(k.cind, 0, n->dims[k.level], ci) : 0) {
      nc = wgrad_lds_chunks(V / (CL_TX * WL_TY * tz), k.cout, k.cind / ci, ch);
      n->part_cap = std::max<int64_t>(n->part_cap, (int64_t)nc * k.cout * 27 * k.cind);
    }
    // the k-split partials of the direct convolution (forward and input gradient)
    n->part_cap = std::max<int64_t>(n->part_cap, (int64_t)conv_splits(V, k.coutp, k.kp) * V * k.cout);
    n->part_cap = std::max<int64_t>(n->part_cap, (int64_t)conv_splits(V, k.rowsb, k.kpb) * V * k.cind);
  }
  const int64_t V0 = vox(n, 0, B);
  {
    int nc;
    int64_t ch;
    wgrad_chunks(V0, 8, pin->widths[0], nc, ch);
    n->part_cap = std::max<int64_t>(n->part_cap, (int64_t)nc * 8 * pin->widths[0]);
  }
  UA(n->stats, stats_cap * 4);
  UA(n->part, n->part_cap * 4);
  UA(n->xin, V0 * 8 * 2);
  for (int l = 0; l < 4; ++l) {
    const int64_t Vn = vox(n, l + 1, B), Vl = vox(n, l, B);
    const int cup = l == 3 ? pin->bottleneck : pin->widths[l + 1];
    UA(n->pool[l], Vn * pin->widths[l] * 2);
    UA(n->gpool[l], Vn * pin->widths[l] * 4);
    UA(n->up[l], Vl * cup * 2);
    UA(n->gcat[l], Vl * (cup + pin->widths[l]) * 4);
  }
  UA(n->hpart, (int64_t)nb256(V0) * 9 * 4);
  UA(n->dlog, V0 * 8 * 2);
  UA(n->y, V0 * pin->cout * 4);
  UA(n->dscal, 16);
#undef UA
  // seeded initial parameters: convolutions and head U(+-1/sqrt(fan_in)),
  // BN scale 1 and shift 0; running statistics mean 0, variance 1
  std::vector<float> h((size_t)n->nparam, 0.f);
  uint64_t ctr = 0;
  auto uni = [&](double bound) {
    uint64_t z = seed + (++ctr) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)(((double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0) * bound);
  };
  for (auto& k : n->blk) {
    const double bnd = 1.0 / std::sqrt(27.0 * k.cin);
    for (int64_t i = 0; i < (int64_t)k.cout * k.cin * 27; ++i) h[(size_t)(k.woff + i)] = uni(bnd);
    for (int c = 0; c < k.cout; ++c) h[(size_t)(k.goff + c)] = 1.f;
  }
  const double hb = 1.0 / std::sqrt((double)pin->widths[0]);
  for (int64_t i = 0; i < (int64_t)pin->cout * pin->widths[0]; ++i) h[(size_t)(n->head_w + i)] = uni(hb);
  for (int o = 0; o < pin->cout; ++o) h[(size_t)(n->head_b + o)] = uni(hb);
  std::vector<float> rsh((size_t)n->nbn * 2, 0.f);
  for (int64_t i = 0; i < n->nbn; ++i) rsh[(size_t)(n->nbn + i)] = 1.f;
  hipError_t e = hipMemcpyAsync(n->theta, h.data(), (size_t)n->nparam * 4, hipMemcpyHostToDevice, n->st);
  if (e == hipSuccess) e = hipMemcpyAsync(rsbuf, rsh.data(), (size_t)n->nbn * 8, hipMemcpyHostToDevice, n->st);
  if (e == hipSuccess) e = hipMemsetAsync(n->am, 0, (size_t)n->nparam * 4, n->st);
  if (e == hipSuccess) e = hipMemsetAsync(n->av, 0, (size_t)n->nparam * 4, n->st);
  if (e == hipSuccess) e = hipStreamSynchronize(n->st);
  if (e != hipSuccess) {
    ufail(nullptr, LBM_EDEVICE, hipGetErrorString(e));
    return bail(LBM_EDEVICE);
  }
  if (int rc = repack(n)) {
    g_unet_err = n->err;
    return bail(rc);
  }
  *out = n;
  return LBM_OK;
}

extern "C" int unet_set_params(unet_net* n, const float* host, int64_t count) {
  if (!n || !host) return ufail(n, LBM_EINVAL, "null argument");
  if (count != n->nparam) return ufail(n, LBM_EINVAL, "parameter count mismatch");
  UCHK(n, hipMemcpyAsync(n->theta, host, (size_t)count * 4, hipMemcpyHostToDevice, n->st));
  if (int rc = repack(n)) return rc;
  UCHK(n, hipStreamSynchronize(n->st));
  return LBM_OK;
}

extern "C" int unet_get_params(unet_net* n, float* host, int64_t count) {
  if (!n || !host) return ufail(n, LBM_EINVAL, "null argument");
  if (count != n->nparam) return ufail(n, LBM_EINVAL, "parameter count mismatch");
  UCHK(n, hipMemcpyAsync(host, n->theta, (size_t)count * 4, hipMemcpyDeviceToHost, n->st));
  UCHK(n, hipStreamSynchronize(n->st));
  return LBM_OK;
}

extern "C" int unet_bn_stats(unet_net* n, float* host, int64_t count) {
  if (!n || !host) return ufail(n, LBM_EINVAL, "null argument");
  if (count != 2 * n->nbn) return ufail(n, LBM_EINVAL, "statistics count mismatch");
  UCHK(n, hipMemcpyAsync(host, n->blk[0].rmean, (size_t)count * 4, hipMemcpyDeviceToHost, n->st));
  UCHK(n, hipStreamSynchronize(n->st));
  return LBM_OK;
}

// A convolution of a block (or its input-gradient adjoint) with rows
// padded output channels: the LDS-tiled kernel where one of its boxes and
// channel chunks applies (inputs in multiples of 32 channels, or the
// 8-channel input layer; the grid in 4 x 4 x 16 or 4 x 8 x 8 boxes), else
// the direct one.  Returns the number of blocks along x, the number of
// per-block statistics partials.
template <int CC, int TY, int TZ>
static void launch_conv_lds(unet_net* n, const ConvArgs& a, int rows, unsigned gx) {
  // 96 rows per block (the input gradients of the decoder's concatenating
  // convolutions): each staged halo value feeds six MFMA row tiles
  if constexpr (CC == 32) {
    if (rows % 96 == 0) {
      hipLaunchKernelGGL((conv_lds_kernel<96, CC, TY, TZ>), dim3(gx, (unsigned)(rows / 96)), dim3(256), 0, n->st, a);
      return;
    }
  }
  if (rows % 64 == 0)
    hipLaunchKernelGGL((conv_lds_kernel<64, CC, TY, TZ>), dim3(gx, (unsigned)(rows / 64)), dim3(256), 0, n->st, a);
  else
    hipLaunchKernelGGL((conv_lds_kernel<32, CC, TY, TZ>), dim3(gx, (unsigned)(rows / 32)), dim3(256), 0, n->st, a);
}

static unsigned conv(unet_net* n, const ConvArgs& a, int rows) {
  const int64_t V = (int64_t)a.B * a.X * a.Y * a.Z;
  const int cc = a.c0 % 32 == 0 && a.c1 % 32 == 0 ? 32 : (a.c0 == 8 && a.c1 == 0 ? 8 : 0);
  const bool box16 = a.X % CL_TX == 0 && a.Y % 4 == 0 && a.Z % 16 == 0;
  const bool box8 = a.X % CL_TX == 0 && a.Y % 8 == 0 && a.Z % 8 == 0;
  if (a.taps == 27 && cc && (box16 || box8)) {
    const unsigned gx = (unsigned)(V / 256);
    if (cc == 32 && box16) launch_conv_lds<32, 4, 16>(n, a, rows, gx);
    else if (cc == 32) launch_conv_lds<32, 8, 8>(n, a, rows, gx);
    else if (box16) launch_conv_lds<8, 4, 16>(n, a, rows, gx);
    else launch_conv_lds<8, 8, 8>(n, a, rows, gx);
    return gx;
  }
  const unsigned gx = (unsigned)((V + CV_VOX - 1) / CV_VOX);
  const int ksteps = a.kp / 32;
  int ks = conv_splits(V, rows, a.kp);
  if (ks > 1) ks = (int)std::min<int64_t>(ks, n->part_cap / (V * a.cout));  // batches below max_batch
  ConvArgs b = a;
  if (ks > 1) {
    const int per = (ksteps + ks - 1) / ks;
    ks = (ksteps + per - 1) / per;
    b.kchunk = 32 * per;
    b.out = n->part;
    b.stats = nullptr;
    hipLaunchKernelGGL(conv_kernel, dim3(gx, (unsigned)(rows / CV_CO), (unsigned)ks), dim3(256), 0, n->st, b);
    const unsigned gr = (unsigned)((V + CSR_VOX - 1) / CSR_VOX);
    hipLaunchKernelGGL(conv_split_reduce_kernel, dim3(gr, (unsigned)((a.cout + 31) / 32)), dim3(256), 0, n->st,
                       n->part, ks, V, a.cout, a.out, a.stats);
    return gr;
  }
  b.kchunk = a.kp;
  hipLaunchKernelGGL(conv_kernel, dim3(gx, (unsigned)(rows / CV_CO)), dim3(256), 0, n->st, b);
  return gx;
}

// one conv-BN-ReLU block forward
static void block_fwd(unet_net* n, Blk& k, int B, const uint16_t* in0, int c0, const uint16_t* in1, int c1,
                      bool train) {
  const int* d = n->dims[k.level];
  const int64_t V = vox(n, k.level, B);
  ConvArgs a{};
  a.in0 = in0; a.in1 = in1; a.c0 = c0; a.c1 = c1;
  a.wt = k.wt; a.kp = k.kp; a.out = k.z; a.cout = k.cout; a.taps = 27;
  a.B = B; a.X = d[0]; a.Y = d[1]; a.Z = d[2];
  a.stats = train ? n->stats : nullptr;
  const unsigned gx = conv(n, a, k.coutp);
  hipLaunchKernelGGL(bn_finalize_kernel, dim3((unsigned)k.cout), dim3(256), 0, n->st, n->stats, (int64_t)gx, k.cout,
                     (double)V, n->theta + k.goff, n->theta + k.boff, k.rmean, k.rvar, k.mean, k.istd, k.scale,
                     k.shift, train ? 1 : 0);
  hipLaunchKernelGGL(bn_relu_kernel, dim3(nb256(V * k.cout / 8)), dim3(256), 0, n->st, k.z, V, k.cout, k.scale,
                     k.shift, k.a);
}

static void run_forward(unet_net* n, const uint16_t* x, int B, bool train) {
  const unet_params& p = n->p;
  const int64_t P = (int64_t)p.nx * p.ny * p.nz;
  hipLaunchKernelGGL(input_kernel, dim3(nb256(B * P)), dim3(256), 0, n->st, x, P, B, p.cin, n->xin);
  for (int l = 0; l < 4; ++l) {
    Blk& ka = n->blk[ienc(l, 0)];
    if (l == 0) block_fwd(n, ka, B, n->xin, 8, nullptr, 0, train);
    else block_fwd(n, ka, B, n->pool[l - 1], p.widths[l - 1], nullptr, 0, train);
    Blk& kb = n->blk[ienc(l, 1)];
    block_fwd(n, kb, B, ka.a, ka.cout, nullptr, 0, train);
    const int* d = n->dims[l];
    const int64_t nout = vox(n, l + 1, B) * kb.cout / 8;
    hipLaunchKernelGGL(maxpool_kernel, dim3(nb256(nout)), dim3(256), 0, n->st, kb.a, B, d[0], d[1], d[2], kb.cout,
                       n->pool[l]);
  }
  block_fwd(n, n->blk[ibot(0)], B, n->pool[3], p.widths[3], nullptr, 0, train);
  block_fwd(n, n->blk[ibot(1)], B, n->blk[ibot(0)].a, p.bottleneck, nullptr, 0, train);
  const Blk* prev = &n->blk[ibot(1)];
  for (int l = 3; l >= 0; --l) {
    const int* dc = n->dims[l + 1];
    const int64_t nout = vox(n, l, B) * prev->cout / 8;
    const int64_t zg = (int64_t)dc[2] * (prev->cout / 8), ny = dc[1], nbx = 2 * (int64_t)B * dc[0];
    if (ny <= 65535 && nbx <= 65535)
      hipLaunchKernelGGL(upsample_block_kernel, dim3((unsigned)((zg + 255) / 256), (unsigned)ny, (unsigned)nbx),
                         dim3(256), 0, n->st, prev->a, B, dc[0], dc[1], dc[2], prev->cout, n->up[l]);
    else
      hipLaunchKernelGGL(upsample_kernel, dim3(nb256(nout)), dim3(256), 0, n->st, prev->a, B, dc[0], dc[1], dc[2],
                         prev->cout, n->up[l]);
    Blk& ka = n->blk[idec(l, 0)];
    block_fwd(n, ka, B, n->up[l], prev->cout, n->blk[ienc(l, 1)].a, p.widths[l], train);
    Blk& kb = n->blk[idec(l, 1)];
    block_fwd(n, kb, B, ka.a, ka.cout, nullptr, 0, train);
    prev = &kb;
  }
}

// head over the last decoder block's activation a: y [B][cout][P] FP32
static void launch_head(unet_net* n, const uint16_t* a, int B, float* y) {
  const unet_params& p = n->p;
  const int64_t P = (int64_t)p.nx * p.ny * p.nz;
  if (p.cout == 4)
    hipLaunchKernelGGL(head_kernel<4>, dim3(nb256(B * P)), dim3(256), 0, n->st, a, P, B, p.widths[0],
                       n->theta + n->head_w, n->theta + n->head_b, p.cout, y);
  else
    hipLaunchKernelGGL(head_kernel<0>, dim3(nb256(B * P)), dim3(256), 0, n->st, a, P, B, p.widths[0],
                       n->theta + n->head_w, n->theta + n->head_b, p.cout, y);
}
static int check_batch(unet_net* n, int B) {
  if (B < 1 || B > n->p.max_batch) return ufail(n, LBM_EINVAL, "batch outside [1, max_batch]");
  return LBM_OK;
}

extern "C" int unet_forward(unet_net* n, const uint16_t* x, int32_t B, int32_t training, float* y) {
  if (!n || !x || !y) return ufail(n, LBM_EINVAL, "null argument");
  if (int rc = check_batch(n, B)) return rc;
  run_forward(n, x, B, training != 0);
  const unet_params& p = n->p;
  const int64_t P = (int64_t)p.nx * p.ny * p.nz;
  launch_head(n, n->blk[idec(0, 1)].a, B, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ufail(n, LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

// weight gradient of a block (or of the head with taps = 1)
static void wgrad(unet_net* n, int level, int B, const uint16_t* dz, int coutp_rows, int cout_param,
                  const uint16_t* in0, int c0, const uint16_t* in1, int c1, int taps, int cin_param, float* dW) {
  const int* d = n->dims[level];
  const int64_t V = vox(n, level, B);
  const int cind = c0 + c1;
  const int K = taps * cind;
  int nchunk;
  int64_t chunk;
  int ci = 0;
  const int tz = taps == 27 && coutp_rows % 32 == 0 ? lds_tiling(c0, c1, d, ci) : 0;
  if (tz) {
    WgradLdsArgs a{};
    a.dz = dz; a.cout = coutp_rows; a.in0 = in0; a.in1 = in1; a.c0 = c0; a.c1 = c1;
    a.B = B; a.X = d[0]; a.Y = d[1]; a.Z = d[2]; a.part = n->part;
    nchunk = wgrad_lds_chunks(V / (CL_TX * WL_TY * tz), coutp_rows, cind / ci, a.per_chunk);
    const dim3 grid((unsigned)nchunk, (unsigned)(coutp_rows / 32), (unsigned)(cind / ci));
    if (ci == 8) hipLaunchKernelGGL((wgrad_lds_kernel<16, 8>), grid, dim3(192), 0, n->st, a);
    else if (tz == 16) hipLaunchKernelGGL((wgrad_lds_kernel<16, 32>), grid, dim3(192), 0, n->st, a);
    else hipLaunchKernelGGL((wgrad_lds_kernel<8, 32>), grid, dim3(192), 0, n->st, a);
    const int64_t ncol = (int64_t)cout_param * K;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((ncol + WR_COLS - 1) / WR_COLS)), dim3(256), 0, n->st,
                       n->part, nchunk, coutp_rows, cout_param, cin_param, cind, taps, dW);
    return;
  }
  wgrad_chunks(V, coutp_rows, K, nchunk, chunk);
  WgradArgs a{};
  a.dz = dz; a.cout = coutp_rows; a.in0 = in0; a.in1 = in1; a.c0 = c0; a.c1 = c1; a.taps = taps;
  a.B = B; a.X = d[0]; a.Y = d[1]; a.Z = d[2]; a.chunk = chunk; a.part = n->part;
  hipLaunchKernelGGL(wgrad_kernel, dim3((unsigned)((coutp_rows + 63) / 64), (unsigned)((K + 63) / 64), (unsigned)nchunk),
                     dim3(256), 0, n->st, a);
  const int64_t ncol = (int64_t)cout_param * K;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((ncol + WR_COLS - 1) / WR_COLS)), dim3(256), 0, n->st,
                     n->part, nchunk, coutp_rows, cout_param, cin_param, cind, taps, dW);
}

// adjoint of one block: from k.g (dL/da) to dL/dz, the parameter gradients
// and (unless gin is null) dL/d(input) FP32 [V][cind] into gin
static void block_bwd(unet_net* n, Blk& k, int B, const uint16_t* in0, int c0, const uint16_t* in1, int c1,
                      float* gin) {
  const int* d = n->dims[k.level];
  const int64_t V = vox(n, k.level, B);
  const int64_t nblk = nb256(V);
  hipLaunchKernelGGL(bn_bwd_reduce_kernel, dim3((unsigned)nblk), dim3(256), 256 * 8 * 2 * sizeof(float), n->st, k.g,
                     k.z, V, k.cout, k.scale, k.shift, k.mean, k.istd, n->stats);
  hipLaunchKernelGGL(bn_bwd_finalize_kernel, dim3((unsigned)k.cout), dim3(256), 0, n->st, n->stats, nblk, k.cout,
                     (double)V, n->theta + k.goff, k.istd, n->grad + k.goff, n->grad + k.boff, k.coef);
  hipLaunchKernelGGL(bn_bwd_apply_kernel, dim3(nb256(V * k.cout / 8)), dim3(256), 0, n->st, k.g, k.z, V, k.cout,
                     k.scale, k.shift, k.mean, k.istd, k.coef, k.dz);
  wgrad(n, k.level, B, k.dz, k.cout, k.cout, in0, c0, in1, c1, 27, k.cin, n->grad + k.woff);
  if (gin) {
    ConvArgs a{};
    a.in0 = k.dz; a.in1 = nullptr; a.c0 = k.cout; a.c1 = 0;
    a.wt = k.wb; a.kp = k.kpb; a.out = gin; a.cout = k.cind; a.taps = 27;
    a.B = B; a.X = d[0]; a.Y = d[1]; a.Z = d[2]; a.stats = nullptr;
    conv(n, a, k.rowsb);
  }
}

extern "C" int unet_loss_grad(unet_net* n, const uint16_t* x, const float* target, const uint8_t* mask, int32_t B,
                              float* loss, float* host_grads) {
  if (!n || !x || !target || !mask) return ufail(n, LBM_EINVAL, "null argument");
  if (int rc = check_batch(n, B)) return rc;
  const unet_params& p = n->p;
  const int64_t P = (int64_t)p.nx * p.ny * p.nz;
  const int64_t V0 = (int64_t)B * P;
  run_forward(n, x, B, true);
  Blk& last = n->blk[idec(0, 1)];
  launch_head(n, last.a, B, n->y);
  // dscal[0]: mask cells, [2]: the loss denominator B * cout * cells, [1]: the loss
  hipLaunchKernelGGL(mask_count_kernel, dim3(1), dim3(1024), 0, n->st, mask, P, (double)B * p.cout, n->dscal);
  if (p.cout == 4 && p.widths[0] == 32)
    hipLaunchKernelGGL((head_bwd_grouped_kernel<4, 4>), dim3(nb256(V0)), dim3(1024), 0, n->st, last.a, n->y, target,
                       mask, n->dscal + 2, P, B, n->theta + n->head_w, last.g, n->dlog, n->hpart);
  else if (p.cout == 4)
    hipLaunchKernelGGL(head_bwd_kernel<4>, dim3(nb256(V0)), dim3(256), 0, n->st, last.a, n->y, target, mask,
                       n->dscal + 2, P, B, p.widths[0], n->theta + n->head_w, p.cout, last.g, n->dlog, n->hpart);
  else
    hipLaunchKernelGGL(head_bwd_kernel<0>, dim3(nb256(V0)), dim3(256), 0, n->st, last.a, n->y, target, mask,
                       n->dscal + 2, P, B, p.widths[0], n->theta + n->head_w, p.cout, last.g, n->dlog, n->hpart);
  hipLaunchKernelGGL(head_reduce_kernel, dim3((unsigned)(1 + p.cout)), dim3(256), 0, n->st, n->hpart,
                     (int64_t)nb256(V0), n->dscal + 2, n->dscal + 1, n->grad + n->head_b);
  wgrad(n, 0, B, n->dlog, 8, p.cout, last.a, p.widths[0], nullptr, 0, 1, p.widths[0], n->grad + n->head_w);
  // decoder, from level 0 up
  for (int l = 0; l < 4; ++l) {
    Blk& kb = n->blk[idec(l, 1)];
    Blk& ka = n->blk[idec(l, 0)];
    block_bwd(n, kb, B, ka.a, ka.cout, nullptr, 0, ka.g);
    const Blk& prev = l == 3 ? n->blk[ibot(1)] : n->blk[idec(l + 1, 1)];
    block_bwd(n, ka, B, n->up[l], prev.cout, n->blk[ienc(l, 1)].a, p.widths[l], n->gcat[l]);
    const int* dc = n->dims[l + 1];
    // one thread per 2 x 2 x 2 block of inputs and 8 channels
    const int64_t nin = (int64_t)B * ((dc[0] + 1) / 2) * ((dc[1] + 1) / 2) * ((dc[2] + 1) / 2) * (prev.cout / 8);
    hipLaunchKernelGGL(upsample_bwd_kernel, dim3(nb256(nin)), dim3(256), 0, n->st, n->gcat[l], prev.cout + p.widths[l],
                       B, dc[0], dc[1], dc[2], prev.cout, n->blk[l == 3 ? ibot(1) : idec(l + 1, 1)].g);
  }
  // bottleneck
  {
    Blk& kb = n->blk[ibot(1)];
    Blk& ka = n->blk[ibot(0)];
    block_bwd(n, kb, B, ka.a, ka.cout, nullptr, 0, ka.g);
    block_bwd(n, ka, B, n->pool[3], p.widths[3], nullptr, 0, n->gpool[3]);
  }
  // encoder, from level 3 down
  for (int l = 3; l >= 0; --l) {
    Blk& kb = n->blk[ienc(l, 1)];
    Blk& ka = n->blk[ienc(l, 0)];
    const int* d = n->dims[l];
    const int cup = l == 3 ? p.bottleneck : p.widths[l + 1];
    const int64_t nout = vox(n, l + 1, B) * kb.cout / 8;
    hipLaunchKernelGGL(maxpool_bwd_kernel, dim3(nb256(nout)), dim3(256), 0, n->st, kb.a, n->gpool[l], B, d[0], d[1],
                       d[2], kb.cout, n->gcat[l], cup + p.widths[l], cup, kb.g);
    block_bwd(n, kb, B, ka.a, ka.cout, nullptr, 0, ka.g);
    if (l == 0) block_bwd(n, ka, B, n->xin, 8, nullptr, 0, nullptr);
    else block_bwd(n, ka, B, n->pool[l - 1], p.widths[l - 1], nullptr, 0, n->gpool[l - 1]);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ufail(n, LBM_EDEVICE, hipGetErrorString(e));
  if (loss) {
    double hs[2] = {0.0, 0.0};
    UCHK(n, hipMemcpyAsync(hs, n->dscal, 16, hipMemcpyDeviceToHost, n->st));
    UCHK(n, hipStreamSynchronize(n->st));
    if (hs[0] == 0.0) return ufail(n, LBM_EINVAL, "empty loss mask");
    *loss = (float)hs[1];
  }
  if (host_grads) {
    UCHK(n, hipMemcpyAsync(host_grads, n->grad, (size_t)n->nparam * 4, hipMemcpyDeviceToHost, n->st));
    UCHK(n, hipStreamSynchronize(n->st));
  }
  return LBM_OK;
}

extern "C" int unet_adam_step(unet_net* n, float lr) {
  if (!n) return ufail(nullptr, LBM_EINVAL, "null argument");
  n->adam_t++;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)n->adam_t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)n->adam_t)));
  hipLaunchKernelGGL(adam_kernel, dim3(nb256(n->nparam)), dim3(256), 0, n->st, n->theta, n->grad, n->am, n->av,
                     n->nparam, lr, (float)b1, (float)b2, c1, c2, 1e-8f);
  return repack(n);
}

extern "C" int unet_train_step(unet_net* n, const uint16_t* x, const float* target, const uint8_t* mask, int32_t B,
                               float lr, float* loss) {
  int rc = unet_loss_grad(n, x, target, mask, B, loss, nullptr);
  if (rc) return rc;
  return unet_adam_step(n, lr);
}

extern "C" void unet_destroy(unet_net* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->st);
  free_unet(n);
  delete n;
}

extern "C" const char* unet_last_error(const unet_net* n) { return n ? n->err.c_str() : g_unet_err.c_str(); }
