// Learned preconditioner for the pressure Poisson solve: a 3D U-Net on the
// node grid of a uniform mesh, evaluated and trained with hand-written
// kernels for gfx950.
//
// Network (4 levels, channels 16/32/48/64, two 3x3x3 conv + ReLU per level
// and side, average pooling down, nearest-neighbour upsampling and channel
// concatenation [upsampled, skip] up, a 1x1x1 convolution to one channel).
// Input channels: 0 = log(1/rho(phi*)) / log(rho+/rho-), 1 = r / rms(r)
// (channels 2..7 are zero padding so that every stored row is 16 bytes).
// As a preconditioner the network N(r) = rms(r) K Net(coef, r / rms(r)) (K a
// fixed output scale stored with the weights) is either used alone or, with
// a damping omega > 0, as the coarse correction between two damped-Jacobi
// sweeps: z1 = omega D^-1 r, r1 = r - A z1, n = N(r1), z2 = z1 + beta n with
// the A-norm-optimal step beta = n.r1 / n.A n along n (either sign),
// z = z2 + omega D^-1 (r - A z2); finally 1^T z = 0.
//
// Storage: activations channels-last (voxel-major) bfloat16; weights FP32
// masters with two bfloat16 copies, [tap][co][ci] for the forward pass and
// [flipped tap][ci][co] for the input gradient.  The 3x3x3 convolutions are
// implicit GEMMs on v_mfma_f32_16x16x32_bf16 (M = voxels, N = output
// channels, K = 27 taps x input channels, FP32 accumulation); the input
// gradient is the same kernel with the flipped, transposed weights; the
// weight gradient (M = input channels, N = output channels, K = voxels)
// stages voxel tiles in LDS and reduces split partial sums in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "chns_internal.h"

namespace chns {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kLayers = 14;
constexpr int kInCh = 8;
constexpr int kCh[4] = {16, 32, 48, 64};
constexpr int kWgradSplits = 48;

struct ULayer {
  int ci = 0, co = 0;
  size_t off = 0;  // offset of W[27][ci][co] in the FP32 parameter vector
  uint16_t* wf = nullptr;
  uint16_t* wb = nullptr;
};

// activations (and their gradients) for one cubic grid edge E
struct UActs {
  int E = 0;
  bool grads = false;
  uint16_t *X = nullptr, *A0 = nullptr, *cat0 = nullptr, *P0 = nullptr, *A2 = nullptr, *cat1 = nullptr,
           *P1 = nullptr, *A4 = nullptr, *cat2 = nullptr, *P2 = nullptr, *A6 = nullptr, *A7 = nullptr,
           *A8 = nullptr, *A9 = nullptr, *A10 = nullptr, *A11 = nullptr, *A12 = nullptr, *A13 = nullptr;
  uint16_t *dA13 = nullptr, *dA12 = nullptr, *dcat0 = nullptr, *dA11 = nullptr, *dA10 = nullptr,
           *dcat1 = nullptr, *dA9 = nullptr, *dA8 = nullptr, *dcat2 = nullptr, *dA7 = nullptr, *dA6 = nullptr,
           *dP2 = nullptr, *dA4 = nullptr, *dP1 = nullptr, *dA2 = nullptr, *dP0 = nullptr, *dA0 = nullptr;
  float *out = nullptr, *target = nullptr, *mask = nullptr, *dout = nullptr;
};

struct UNet {
  ULayer L[kLayers];
  size_t nparam = 0;   // 3x3x3 weights of all layers, then w_out[16]
  size_t wout_off = 0;
  float* W = nullptr;  // FP32 masters
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  uint16_t* wbf = nullptr;
  float K = 1.0f;
  float omega = 0.0f;  // Jacobi damping of the smoothing sweeps (0: network alone)
  int step = 0;
  bool ready = false;
  std::vector<UActs> acts;
  float* partial = nullptr;
  size_t partial_cap = 0;
  double* red = nullptr;      // reduction partials (device)
  double* scal = nullptr;     // device scalars: [0] rms, [1] mean, [2] loss or beta, [3] count,
                              // [4..7] A-norm objective, [8] n.A n, [9] g.n
  double* scal_host = nullptr;
  float* gout_part = nullptr;  // w_out gradient partials
  double *zb = nullptr, *qb = nullptr;  // node vectors of the A-norm objective
  double* tb[10] = {};                  // training work vectors (smoothing)
  double* hb64[4] = {};                 // preconditioner work vectors
  float* hb32[4] = {};
  // adaptive meshes: the network runs on the uniform node grid of level
  // kGridLevel; P (mesh nodes <- grid), R = P^T and Q (grid <- mesh nodes)
  bool grid_built = false;
  int64_t n_grid = 0;
  int32_t *gP_ptr = nullptr, *gP_col = nullptr, *gR_ptr = nullptr, *gR_col = nullptr, *gQ_ptr = nullptr,
          *gQ_col = nullptr;
  double *gP_val = nullptr, *gR_val = nullptr, *gQ_val = nullptr;
  double* phig = nullptr;  // phi~ sampled at the grid points
  double* xg64[2] = {};    // grid residual and network output
  float* xg32[2] = {};
};

namespace {

constexpr int kT = 256;
constexpr int kRedBlocks = 1024;
// level of the uniform node grid (129^3 points) the network sees on adaptive
// meshes: the level it is trained on
constexpr int kGridLevel = 7;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf(u32x4 t) { return __builtin_bit_cast(bf16x8, t); }

// fixed-order sum of part[0 .. np) (stride `step`) by one block of 256
// threads; every thread returns the total
__device__ double block_total(const double* part, int np, double* sh, int step = 1) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) v += part[(int64_t)i * step];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

#define ULOOP(i, n) for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

inline unsigned nblk(int64_t n) {
  int64_t g = (n + kT - 1) / kT;
  if (g > 65535) g = 65535;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------- convolution
// out[v][n] = sum_tap sum_k in[v + off(tap)][k] wt[tap][n][k], zero outside
// the E^3 grid; n < 16 NB, k < ci (implicit GEMM: M = voxels, N = output
// channels, K = 27 taps x input channels in chunks of 32, one MFMA per
// 16-voxel row block, column block and chunk).
// The input is staged in LDS: a workgroup (four waves)
// owns an output tile of 4 (z) x 4 (y) x 16 (x) voxels; per chunk of 32 input
// channels the (4+2) x (4+2) x (16+2) halo is loaded once (16-byte rows,
// zero outside the grid and beyond ci) and the 27 taps read it from LDS.
// Wave w computes the z-slice w of the tile: four 16-voxel rows (one per y)
// times NB 16-channel column blocks.
constexpr int kTX = 16, kTY = 4, kTZ = 4;

// Output tile of a convolution workgroup.  Workgroups are dealt round-robin
// to the 8 XCDs (linear id b on XCD b % 8, each XCD with its own L2); the
// linear id is remapped so that each XCD runs a contiguous run of tiles (a
// slab of the grid), whose overlapping halos then meet in one L2.
__device__ __forceinline__ void conv_tile(int& ox, int& oy, int& oz) {
  constexpr uint32_t kXcd = 8;
  const uint32_t gx = gridDim.x, gy = gridDim.y, g = gx * gy * gridDim.z;
  const uint32_t b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const uint32_t per = g / kXcd, rem = g % kXcd, x = b % kXcd;
  const uint32_t t = x * per + (x < rem ? x : rem) + b / kXcd;
  ox = (int)(t % gx) * kTX;
  oy = (int)((t / gx) % gy) * kTY;
  oz = (int)(t / (gx * gy)) * kTZ;
}
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHRow = 40;  // bf16 per halo voxel: 32 channels + 8 padding (bank spread)
template <int NB>
__global__ __launch_bounds__(256) void k_conv3_tile(const uint16_t* __restrict__ in, int cs_in, int ci,
                                                    const uint16_t* __restrict__ wt, uint16_t* __restrict__ out,
                                                    int cs_out, int E, int relu) {
  __shared__ __attribute__((aligned(16))) uint16_t H[kHZ * kHY * kHX * kHRow];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int co = NB * 16;
  int ox, oy, oz;
  conv_tile(ox, oy, oz);
  f32x4 acc[4][NB];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nchunk = (ci + 31) >> 5;
  for (int c = 0; c < nchunk; ++c) {
    // stage the halo of this channel chunk: 4 rows of 16 bytes per voxel;
    // a thread issues all its loads before its first LDS store
    constexpr int NS = kHZ * kHY * kHX * 4, NJ = (NS + 255) / 256;
    u32x4 t[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int i = tid + j * 256;
      const int hv = i >> 2, part = i & 3;
      const int hx = hv % kHX, hy = (hv / kHX) % kHY, hz = hv / (kHX * kHY);
      const int x = ox + hx - 1, y = oy + hy - 1, z = oz + hz - 1;
      const int k = c * 32 + part * 8;
      t[j] = u32x4{0u, 0u, 0u, 0u};
      if (i < NS && k < ci && x >= 0 && x < E && y >= 0 && y < E && z >= 0 && z < E)
        t[j] = *(const u32x4*)(in + ((int64_t)(z * E + y) * E + x) * cs_in + k);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int i = tid + j * 256;
      if (i < NS) *(u32x4*)&H[(i >> 2) * kHRow + (i & 3) * 8] = t[j];
    }
    __syncthreads();
    const int k0 = c * 32 + g * 8;
    const bool kin = k0 < ci;
    if constexpr (NB <= 2) {
      // few output channels: an activation fragment feeds only NB MFMAs, so
      // LDS bandwidth bounds the loop.  Per dz, the 9 taps' weights stay in
      // registers and each halo row (hy, dx) is read once for the up to
      // three output rows it serves (mb = hy - 1 - dy): 18 LDS reads for 36
      // MFMAs per NB instead of 36
#pragma unroll 1
      for (int dz = -1; dz <= 1; ++dz) {
        u32x4 w[9][NB];
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            w[t][nb] = u32x4{0u, 0u, 0u, 0u};
            if (kin) w[t][nb] = *(const u32x4*)(wt + ((int64_t)((dz + 1) * 9 + t) * co + nb * 16 + r16) * ci + k0);
          }
        const int hz = wave + 1 + dz;
#pragma unroll
        for (int hy = 0; hy < kTY + 2; ++hy) {
          // one halo row's reads at a time (bounds the registers in flight)
          asm volatile("" ::: "memory");
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const u32x4 ta = *(const u32x4*)&H[((hz * kHY + hy) * kHX + r16 + 1 + dx) * kHRow + g * 8];
            const bf16x8 av = as_bf(ta);
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
              const int mb = hy - 1 - dy;
              if (mb < 0 || mb >= kTY) continue;
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, as_bf(w[(dy + 1) * 3 + dx + 1][nb]),
                                                                     acc[mb][nb], 0, 0, 0);
            }
          }
        }
      }
      __syncthreads();
      continue;
    }
    // weight fragments of a group of taps are loaded together (one latency
    // per group instead of one per tap)
    constexpr int TG = 3;
    for (int t0 = 0; t0 < 27; t0 += TG) {
      u32x4 w[TG][NB];
#pragma unroll
      for (int t = 0; t < TG; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          w[t][nb] = u32x4{0u, 0u, 0u, 0u};
          if (kin) w[t][nb] = *(const u32x4*)(wt + ((int64_t)(t0 + t) * co + nb * 16 + r16) * ci + k0);
        }
#pragma unroll
      for (int t = 0; t < TG; ++t) {
        const int tap = t0 + t;
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        const int hz = wave + 1 + dz, hx = r16 + 1 + dx;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const int hy = mb + 1 + dy;
          const u32x4 ta = *(const u32x4*)&H[((hz * kHY + hy) * kHX + hx) * kHRow + g * 8];
          const bf16x8 av = as_bf(ta);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, as_bf(w[t][nb]), acc[mb][nb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // lane holds rows 4 g + r (x offsets) of column r16 (channel) of each block
  const int z = oz + wave;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int y = oy + mb;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = ox + 4 * g + r;
      if (x >= E || y >= E || z >= E) continue;
      const int64_t v = (int64_t)(z * E + y) * E + x;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        float val = acc[mb][nb][r];
        if (relu) val = fmaxf(val, 0.0f);
        out[v * cs_out + nb * 16 + r16] = f2bf(val);
      }
    }
  }
}

// Small input-channel counts (ci = 8, 16, 32; 48 with 48 output channels,
// where the 73 KB halo still leaves enough occupancy): the whole halo (all
// channels) fits in LDS, and K = 27 taps x ci is one flat dimension, k = tap ci + c, cut
// into chunks of 32 that may span several taps (each 8-lane group of a
// fragment reads its own tap), so the MFMAs carry no zero padding.
template <int NB, int CI>
__global__ __launch_bounds__(256) void k_conv3_flat(const uint16_t* __restrict__ in, int cs_in,
                                                    const uint16_t* __restrict__ wt, uint16_t* __restrict__ out,
                                                    int cs_out, int E, int relu) {
  constexpr int ROW = CI + 8;  // bf16 per halo voxel (8 padding: bank spread, 16-byte rows)
  constexpr int PARTS = CI / 8;
  constexpr int KT = 27 * CI;
  constexpr int NQ = (KT + 31) / 32;
  constexpr int QG = NB <= 1 ? NQ : (NB <= 2 ? 9 : 3);  // chunks whose weights load together
  __shared__ __attribute__((aligned(16))) uint16_t H[kHZ * kHY * kHX * ROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int co = NB * 16;
  int ox, oy, oz;
  conv_tile(ox, oy, oz);
  if constexpr (CI >= 32) {
    // all loads of a thread before its first LDS store (measured faster
    // for 32 and 48 channels; for 16 the unrolled loads cost occupancy); the
    // fence keeps the weight loads below out of this phase
    constexpr int NS = kHZ * kHY * kHX * PARTS, NJ = (NS + 255) / 256;
    u32x4 t[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int i = tid + j * 256;
      const int hv = i / PARTS, part = i % PARTS;
      const int hx = hv % kHX, hy = (hv / kHX) % kHY, hz = hv / (kHX * kHY);
      const int x = ox + hx - 1, y = oy + hy - 1, z = oz + hz - 1;
      t[j] = u32x4{0u, 0u, 0u, 0u};
      if (i < NS && x >= 0 && x < E && y >= 0 && y < E && z >= 0 && z < E)
        t[j] = *(const u32x4*)(in + ((int64_t)(z * E + y) * E + x) * cs_in + part * 8);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int i = tid + j * 256;
      if (i < NS) *(u32x4*)&H[(i / PARTS) * ROW + (i % PARTS) * 8] = t[j];
    }
    asm volatile("" ::: "memory");
  } else {
    for (int i = tid; i < kHZ * kHY * kHX * PARTS; i += 256) {
      const int hv = i / PARTS, part = i % PARTS;
      const int hx = hv % kHX, hy = (hv / kHX) % kHY, hz = hv / (kHX * kHY);
      const int x = ox + hx - 1, y = oy + hy - 1, z = oz + hz - 1;
      u32x4 t = {0u, 0u, 0u, 0u};
      if (x >= 0 && x < E && y >= 0 && y < E && z >= 0 && z < E)
        t = *(const u32x4*)(in + ((int64_t)(z * E + y) * E + x) * cs_in + part * 8);
      *(u32x4*)&H[hv * ROW + part * 8] = t;
    }
  }
  __syncthreads();
  f32x4 acc[4][NB];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int q0 = 0; q0 < NQ; q0 += QG) {
    u32x4 w[QG][NB];
#pragma unroll
    for (int qq = 0; qq < QG; ++qq) {
      const int k = (q0 + qq) * 32 + g * 8;
      const int tap = k / CI, c = k % CI;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        w[qq][nb] = u32x4{0u, 0u, 0u, 0u};
        if (q0 + qq < NQ && k < KT) w[qq][nb] = *(const u32x4*)(wt + ((int64_t)tap * co + nb * 16 + r16) * CI + c);
      }
    }
#pragma unroll
    for (int qq = 0; qq < QG; ++qq) {
      if (q0 + qq >= NQ) break;
      const int k = (q0 + qq) * 32 + g * 8;
      const bool kin = k < KT;
      const int tap = kin ? k / CI : 0, c = k % CI;
      const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
      const int hz = wave + 1 + dz, hx = r16 + 1 + dx;
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const int hy = mb + 1 + dy;
        u32x4 ta = {0u, 0u, 0u, 0u};
        if (kin) ta = *(const u32x4*)&H[((hz * kHY + hy) * kHX + hx) * ROW + c];
        const bf16x8 av = as_bf(ta);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, as_bf(w[qq][nb]), acc[mb][nb], 0, 0, 0);
      }
    }
  }
  const int z = oz + wave;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int y = oy + mb;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = ox + 4 * g + r;
      if (x >= E || y >= E || z >= E) continue;
      const int64_t v = (int64_t)(z * E + y) * E + x;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        float val = acc[mb][nb][r];
        if (relu) val = fmaxf(val, 0.0f);
        out[v * cs_out + nb * 16 + r16] = f2bf(val);
      }
    }
  }
}

// Weight gradient, one tap per block row: partial[s][tap][i][j] =
// sum over this split's voxels v of in[v + off(tap)][i] dy[v][j]
// (i < 16 MB input channels, zero beyond ci; j < 16 NB output channels).
template <int MB, int NB>
__global__ __launch_bounds__(64) void k_wgrad(const uint16_t* __restrict__ in, int cs_in, int ci,
                                              const uint16_t* __restrict__ dy, int cs_dy, int E, int S,
                                              float* __restrict__ partial) {
  constexpr int CI = MB * 16, CO = NB * 16;
  __shared__ __attribute__((aligned(16))) uint16_t Xs[32][CI + 8];
  __shared__ __attribute__((aligned(16))) uint16_t Ys[32][CO + 8];
  const int lane = threadIdx.x, r16 = lane & 15, g = lane >> 4;
  const int tap = blockIdx.y, s = blockIdx.x;
  const int dz = tap / 9 - 1, dy_ = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const int V = E * E * E;
  f32x4 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nq = (V + 31) / 32;
  for (int q = s; q < nq; q += S) {
    const int v0 = q * 32;
    for (int i = lane; i < 32 * NB * 2; i += 64) {
      const int j = i / (NB * 2), c8 = (i % (NB * 2)) * 8;
      const int v = v0 + j;
      u32x4 t = {0u, 0u, 0u, 0u};
      if (v < V) t = *(const u32x4*)(dy + (int64_t)v * cs_dy + c8);
      *(u32x4*)&Ys[j][c8] = t;
    }
    for (int i = lane; i < 32 * MB * 2; i += 64) {
      const int j = i / (MB * 2), c8 = (i % (MB * 2)) * 8;
      const int v = v0 + j;
      u32x4 t = {0u, 0u, 0u, 0u};
      if (v < V && c8 < ci) {
        const int x = v % E + dx, y = (v / E) % E + dy_, z = v / (E * E) + dz;
        if (x >= 0 && x < E && y >= 0 && y < E && z >= 0 && z < E)
          t = *(const u32x4*)(in + ((int64_t)(z * E + y) * E + x) * cs_in + c8);
      }
      *(u32x4*)&Xs[j][c8] = t;
    }
    __syncthreads();
    bf16x8 a[MB], b[NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      u32x4 t;
#pragma unroll
      for (int h = 0; h < 4; ++h)
        t[h] = (uint32_t)Xs[8 * g + 2 * h][mb * 16 + r16] | ((uint32_t)Xs[8 * g + 2 * h + 1][mb * 16 + r16] << 16);
      a[mb] = as_bf(t);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      u32x4 t;
#pragma unroll
      for (int h = 0; h < 4; ++h)
        t[h] = (uint32_t)Ys[8 * g + 2 * h][nb * 16 + r16] | ((uint32_t)Ys[8 * g + 2 * h + 1][nb * 16 + r16] << 16);
      b[nb] = as_bf(t);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
    __syncthreads();
  }
  float* p = partial + ((int64_t)s * 27 + tap) * CI * CO;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) p[(mb * 16 + 4 * g + r) * CO + nb * 16 + r16] = acc[mb][nb][r];
}

// grad[t][i][j] (+)= sum_s partial[s][t][i][j], fixed order over s
__global__ void k_wgrad_reduce(const float* partial, int S, int ci, int co, int CI, int CO, float* grad,
                               float scale, int accumulate) {
  ULOOP(idx, (int64_t)27 * ci * co) {
    const int j = (int)(idx % co), i = (int)((idx / co) % ci), t = (int)(idx / ((int64_t)ci * co));
    float sum = 0.0f;
    for (int s = 0; s < S; ++s) sum += partial[(((int64_t)s * 27 + t) * CI + i) * CO + j];
    grad[idx] = (accumulate ? grad[idx] : 0.0f) + scale * sum;
  }
}

// ------------------------------------------------------- other layers
// The pooling, upsampling and ReLU-mask kernels work on 8-channel groups
// (16-byte rows; channel counts and channel offsets are multiples of 8).
__device__ __forceinline__ void unpack8(u32x4 t, float* f) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    f[2 * h] = bf2f((uint16_t)(t[h] & 0xFFFFu));
    f[2 * h + 1] = bf2f((uint16_t)(t[h] >> 16));
  }
}
__device__ __forceinline__ u32x4 pack8(const float* f) {
  u32x4 t;
#pragma unroll
  for (int h = 0; h < 4; ++h) t[h] = (uint32_t)f2bf(f[2 * h]) | ((uint32_t)f2bf(f[2 * h + 1]) << 16);
  return t;
}

// P[z][y][x][c] = mean of the 2x2x2 children (coarse edge Ec)
__global__ void k_pool(const uint16_t* in, int cs_in, uint16_t* out, int C, int Ec) {
  const int G = C / 8;
  const int64_t n = (int64_t)Ec * Ec * Ec * G;
  const int Ef = 2 * Ec;
  ULOOP(idx, n) {
    const int grp = (int)(idx % G);
    const int p = (int)(idx / G);
    const int x = p % Ec, y = (p / Ec) % Ec, z = p / (Ec * Ec);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 8; ++k) {
      const int fz = 2 * z + (k >> 2), fy = 2 * y + ((k >> 1) & 1), fx = 2 * x + (k & 1);
      float f[8];
      unpack8(*(const u32x4*)(in + ((int64_t)(fz * Ef + fy) * Ef + fx) * cs_in + grp * 8), f);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += f[j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] *= 0.125f;
    *(u32x4*)(out + (int64_t)p * C + grp * 8) = pack8(s);
  }
}
// dskip[v][c] += dP[parent(v)][c] / 8 (fine edge Ef)
__global__ void k_pool_bwd_add(const uint16_t* dP, int C, uint16_t* dskip, int cs, int Ef) {
  const int G = C / 8;
  const int64_t n = (int64_t)Ef * Ef * Ef * G;
  const int Ec = Ef / 2;
  ULOOP(idx, n) {
    const int grp = (int)(idx % G);
    const int v = (int)(idx / G);
    const int x = v % Ef, y = (v / Ef) % Ef, z = v / (Ef * Ef);
    const int64_t p = ((int64_t)(z / 2) * Ec + y / 2) * Ec + x / 2;
    uint16_t* d = dskip + (int64_t)v * cs + grp * 8;
    float a[8], b[8];
    unpack8(*(const u32x4*)d, a);
    unpack8(*(const u32x4*)(dP + p * C + grp * 8), b);
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = a[j] + b[j] * 0.125f;
    *(u32x4*)d = pack8(a);
  }
}
// out[v][c] (stride cs_out) = in[parent(v)][c] (fine edge Ef)
__global__ void k_up(const uint16_t* in, int C, uint16_t* out, int cs_out, int Ef) {
  const int G = C / 8;
  const int64_t n = (int64_t)Ef * Ef * Ef * G;
  const int Ec = Ef / 2;
  ULOOP(idx, n) {
    const int grp = (int)(idx % G);
    const int v = (int)(idx / G);
    const int x = v % Ef, y = (v / Ef) % Ef, z = v / (Ef * Ef);
    const int64_t p = ((int64_t)(z / 2) * Ec + y / 2) * Ec + x / 2;
    *(u32x4*)(out + (int64_t)v * cs_out + grp * 8) = *(const u32x4*)(in + p * C + grp * 8);
  }
}
// out[p][c] = sum of d[child][c] (stride cs), coarse edge Ec
__global__ void k_up_bwd(const uint16_t* d, int cs, uint16_t* out, int C, int Ec) {
  const int G = C / 8;
  const int64_t n = (int64_t)Ec * Ec * Ec * G;
  const int Ef = 2 * Ec;
  ULOOP(idx, n) {
    const int grp = (int)(idx % G);
    const int p = (int)(idx / G);
    const int x = p % Ec, y = (p / Ec) % Ec, z = p / (Ec * Ec);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 8; ++k) {
      const int fz = 2 * z + (k >> 2), fy = 2 * y + ((k >> 1) & 1), fx = 2 * x + (k & 1);
      float f[8];
      unpack8(*(const u32x4*)(d + ((int64_t)(fz * Ef + fy) * Ef + fx) * cs + grp * 8), f);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += f[j];
    }
    *(u32x4*)(out + (int64_t)p * C + grp * 8) = pack8(s);
  }
}
// dy = dy * (a > 0)
__global__ void k_relu_bwd(uint16_t* dy, int cs_dy, const uint16_t* a, int cs_a, int C, int64_t V) {
  const int G = C / 8;
  ULOOP(idx, V * G) {
    const int grp = (int)(idx % G);
    const int64_t v = idx / G;
    u32x4 t = *(const u32x4*)(dy + v * cs_dy + grp * 8);
    const u32x4 m = *(const u32x4*)(a + v * cs_a + grp * 8);
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      uint32_t w = t[h];
      // bf16 a > 0: sign bit clear and not zero
      if ((m[h] & 0x8000u) || (m[h] & 0x7FFFu) == 0u) w &= 0xFFFF0000u;
      if ((m[h] & 0x80000000u) || (m[h] & 0x7FFF0000u) == 0u) w &= 0x0000FFFFu;
      t[h] = w;
    }
    *(u32x4*)(dy + v * cs_dy + grp * 8) = t;
  }
}

// out[v] = sum_c w[c] a[v][c]
__global__ void k_out(const uint16_t* a, const float* w, float* out, int64_t V) {
  ULOOP(v, V) {
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 16; ++c) s += w[c] * bf2f(a[v * 16 + c]);
    out[v] = s;
  }
}
// loss partials and dout = 2 (out - t) mask / count
__global__ __launch_bounds__(kT) void k_mse(const float* out, const float* t, const float* mask, int64_t V,
                                           double* part) {
  __shared__ double sh[2][4];
  double l = 0.0, c = 0.0;
  ULOOP(v, V) {
    const double d = ((double)out[v] - (double)t[v]) * mask[v];
    l += d * d;
    c += mask[v];
  }
  for (int o = 32; o > 0; o >>= 1) {
    l += __shfl_xor(l, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = l;
    sh[1][threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[blockIdx.x] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    part[kRedBlocks + blockIdx.x] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
  }
}
__global__ __launch_bounds__(256) void k_sum2(const double* part, int np, double* out) {
  __shared__ double sh[4];
  const double a = block_total(part, np, sh), b = block_total(part + kRedBlocks, np, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}
__global__ void k_dout(const float* out, const float* t, const float* mask, const double* lc, float* dout,
                       int64_t V) {
  const float inv = (float)(2.0 / lc[1]);
  ULOOP(v, V) dout[v] = (out[v] - t[v]) * mask[v] * inv;
}
// dA13[v][c] = w[c] dout[v]; partial w_out gradient per block
__global__ __launch_bounds__(kT) void k_out_bwd(const uint16_t* a, const float* w, const float* dout, int64_t V,
                                               uint16_t* da, float* gpart) {
  __shared__ float sh[16][kT / 64];
  float g[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) g[c] = 0.0f;
  ULOOP(v, V) {
    const float d = dout[v];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      da[v * 16 + c] = f2bf(w[c] * d);
      g[c] += bf2f(a[v * 16 + c]) * d;
    }
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    float t = g[c];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) sh[c][threadIdx.x >> 6] = t;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int c = threadIdx.x;
    gpart[blockIdx.x * 16 + c] = (sh[c][0] + sh[c][1]) + (sh[c][2] + sh[c][3]);
  }
}
__global__ __launch_bounds__(256) void k_gout_reduce(const float* gpart, int nb, float* grad, float scale,
                                                     int accumulate) {
  __shared__ float sh[16][4];
  for (int c = 0; c < 16; ++c) {
    float v = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 256) v += gpart[b * 16 + c];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[c][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int c = threadIdx.x;
    const float t = (sh[c][0] + sh[c][1]) + (sh[c][2] + sh[c][3]);
    grad[c] = (accumulate ? grad[c] : 0.0f) + scale * t;
  }
}

// bf16 copies of the FP32 masters in the two layouts
__global__ void k_prep_weights(const float* W, int ci, int co, uint16_t* wf, uint16_t* wb) {
  ULOOP(idx, (int64_t)27 * ci * co) {
    const int o = (int)(idx % co), i = (int)((idx / co) % ci), t = (int)(idx / ((int64_t)ci * co));
    const uint16_t h = f2bf(W[idx]);
    wf[((int64_t)t * co + o) * ci + i] = h;
    wb[((int64_t)(26 - t) * ci + i) * co + o] = h;
  }
}
__global__ void k_adam(float* W, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  ULOOP(i, n) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    W[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ------------------------------------------------------------- packing
// sum of squares of r (partials), for rms(r)
template <typename T>
__global__ __launch_bounds__(kT) void k_sumsq(const T* r, int64_t n, double* part) {
  __shared__ double sh[4];
  double s = 0.0;
  ULOOP(i, n) s += (double)r[i] * (double)r[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
// rms = sqrt(sum / n) into scal[0]
__global__ __launch_bounds__(256) void k_rms(const double* part, int np, int64_t n, double* scal) {
  __shared__ double sh[4];
  const double s = block_total(part, np, sh);
  if (threadIdx.x == 0) scal[0] = s > 0.0 ? sqrt(s / (double)n) : 1.0;
}

// y = M x for a CSR matrix with FP64 values, summed in FP64 in row order
template <typename T>
__global__ void k_csr_apply(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, const T* __restrict__ x, T* __restrict__ y, int64_t rows) {
  ULOOP(i, rows) {
    double acc = 0.0;
    for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) acc += val[k] * (double)x[col[k]];
    y[i] = (T)acc;
  }
}

struct PackGeo {
  int side;            // nodes per axis - 1
  int E;               // grid edge in voxels
  int ox, oy, oz;      // crop origin (nodes)
  int flip;            // bit d mirrors axis d inside the crop
};
__device__ __forceinline__ int64_t voxel_node(const PackGeo& g, int64_t v) {
  int x = (int)(v % g.E), y = (int)((v / g.E) % g.E), z = (int)(v / ((int64_t)g.E * g.E));
  if (g.flip & 1) x = g.E - 1 - x;
  if (g.flip & 2) y = g.E - 1 - y;
  if (g.flip & 4) z = g.E - 1 - z;
  x += g.ox;
  y += g.oy;
  z += g.oz;
  if (x > g.side || y > g.side || z > g.side) return -1;
  const int64_t s1 = g.side + 1;
  return x + s1 * (y + s1 * (int64_t)z);
}
// network input (and training target / mask)
template <typename T>
__global__ void k_pack(PackGeo geo, const double* phi, const T* r, const double* e, const double* scal,
                       double alpha, double beta, double inv_lratio, float K, uint16_t* X, float* target,
                       float* mask) {
  const int64_t V = (int64_t)geo.E * geo.E * geo.E;
  const double rinv = 1.0 / scal[0];
  ULOOP(v, V) {
    const int64_t i = voxel_node(geo, v);
    float c0 = 0.0f, c1 = 0.0f, tg = 0.0f, mk = 0.0f;
    if (i >= 0) {
      const double p = fmin(fmax(phi[i], -1.0), 1.0);
      const double rho = alpha * p + beta;
      c0 = (float)(-log(rho) * inv_lratio);
      c1 = (float)((double)r[i] * rinv);
      if (e) tg = (float)(e[i] * rinv / (double)K);
      mk = 1.0f;
    }
    u32x4 lo = {(uint32_t)f2bf(c0) | ((uint32_t)f2bf(c1) << 16), 0u, 0u, 0u};
    *(u32x4*)(X + v * kInCh) = lo;
    if (target) {
      target[v] = tg;
      mask[v] = mk;
    }
  }
}
// z[node] = rms K sum_c w[c] a13[v][c] for every voxel that is a node
template <typename T>
__global__ void k_unpack(PackGeo geo, const uint16_t* a, const float* w, const double* scal, float K, T* z) {
  const int64_t V = (int64_t)geo.E * geo.E * geo.E;
  const double sc = scal[0] * (double)K;
  ULOOP(v, V) {
    const int64_t i = voxel_node(geo, v);
    if (i < 0) continue;
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 16; ++c) s += w[c] * bf2f(a[v * 16 + c]);
    z[i] = (T)(sc * (double)s);
  }
}
template <typename T>
__global__ __launch_bounds__(kT) void k_sum_part(const T* z, int64_t n, double* part) {
  __shared__ double sh[4];
  double s = 0.0;
  ULOOP(i, n) s += (double)z[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
__global__ __launch_bounds__(256) void k_mean(const double* part, int np, int64_t n, double* scal) {
  __shared__ double sh[4];
  const double s = block_total(part, np, sh);
  if (threadIdx.x == 0) scal[1] = s / (double)n;
}
template <typename T>
__global__ void k_sub(T* z, int64_t n, const double* scal) {
  const double m = scal[1];
  ULOOP(i, n) z[i] = (T)((double)z[i] - m);
}

// A-norm objective on the node grid: partial z.q, z.r, e.r
__global__ __launch_bounds__(kT) void k_dot3(const double* z, const double* q, const double* r, const double* e,
                                            int64_t n, double* part) {
  __shared__ double sh[3][4];
  double a = 0.0, b = 0.0, c = 0.0;
  ULOOP(i, n) {
    a += z[i] * q[i];
    b += z[i] * r[i];
    c += e[i] * r[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = a;
    sh[1][threadIdx.x >> 6] = b;
    sh[2][threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x < 3) part[threadIdx.x * kRedBlocks + blockIdx.x] =
      (sh[threadIdx.x][0] + sh[threadIdx.x][1]) + (sh[threadIdx.x][2] + sh[threadIdx.x][3]);
}
// scal[4..6] = totals; scal[7] = loss (z.q - 2 z.r + e.r) / e.r
__global__ __launch_bounds__(256) void k_fin3(const double* part, int np, double* scal) {
  __shared__ double sh[4];
  double t[3];
  for (int k = 0; k < 3; ++k) t[k] = block_total(part + k * kRedBlocks, np, sh);
  if (threadIdx.x != 0) return;
  scal[4] = t[0];
  scal[5] = t[1];
  scal[6] = t[2];
  scal[7] = t[2] > 0.0 ? (t[0] - 2.0 * t[1] + t[2]) / t[2] : 0.0;
}
// g = dL/dz = 2 (q - r) / e.r
__global__ void k_grad_anorm(const double* q, const double* r, const double* scal, double* g, int64_t n) {
  const double f = scal[6] > 0.0 ? 2.0 / scal[6] : 0.0;
  ULOOP(i, n) g[i] = f * (q[i] - r[i]);
}
// dL/dout at every voxel: rms K g[node] (zero off the grid)
__global__ void k_dout_nodes(PackGeo geo, const double* g, const double* scal, float K, float* dout) {
  const int64_t V = (int64_t)geo.E * geo.E * geo.E;
  const double f = scal[0] * (double)K;
  ULOOP(v, V) {
    const int64_t i = voxel_node(geo, v);
    dout[v] = i < 0 ? 0.0f : (float)(f * g[i]);
  }
}
// smoothing sweeps
template <typename T>
__global__ void k_wdinv(T* out, double w, const T* d, const T* x, int64_t n) {
  ULOOP(i, n) out[i] = (T)(w * (double)d[i] * (double)x[i]);
}
template <typename T>
__global__ void k_rsub(T* t, const T* r, int64_t n) { ULOOP(i, n) t[i] = r[i] - t[i]; }
template <typename T>
__global__ void k_addv(T* z, const T* a, int64_t n) { ULOOP(i, n) z[i] += a[i]; }
// z += w D^-1 (r - t)
template <typename T>
__global__ void k_jcorr(T* z, double w, const T* d, const T* r, const T* t, int64_t n) {
  ULOOP(i, n) z[i] = (T)((double)z[i] + w * (double)d[i] * ((double)r[i] - (double)t[i]));
}
// g -= w q (q = A D^-1 g)
__global__ void k_axpy_neg(double* g, double w, const double* q, int64_t n) { ULOOP(i, n) g[i] -= w * q[i]; }
// out = r - a
template <typename T>
__global__ void k_diffv(T* out, const T* r, const T* a, int64_t n) { ULOOP(i, n) out[i] = r[i] - a[i]; }
// partial a.b (row 0) and a.c (row 1)
template <typename T>
__global__ __launch_bounds__(kT) void k_dot2(const T* a, const T* b, const T* c, int64_t n, double* part) {
  __shared__ double sh[2][4];
  double x = 0.0, y = 0.0;
  ULOOP(i, n) {
    x += (double)a[i] * (double)b[i];
    y += (double)a[i] * (double)c[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    x += __shfl_xor(x, o, 64);
    y += __shfl_xor(y, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = x;
    sh[1][threadIdx.x >> 6] = y;
  }
  __syncthreads();
  if (threadIdx.x < 2)
    part[threadIdx.x * kRedBlocks + blockIdx.x] =
        (sh[threadIdx.x][0] + sh[threadIdx.x][1]) + (sh[threadIdx.x][2] + sh[threadIdx.x][3]);
}
// scal[2] = beta = (n.r1) / (n.A n), the A-norm-optimal step along n (either
// sign; 0 if n.A n is not positive); scal[8] = n.A n
__global__ __launch_bounds__(256) void k_beta(const double* part, int np, double* scal) {
  __shared__ double sh[4];
  const double a = block_total(part, np, sh), b = block_total(part + kRedBlocks, np, sh);
  if (threadIdx.x != 0) return;
  scal[2] = b > 0.0 ? a / b : 0.0;
  scal[8] = b;
}
// z = z1 + beta z (z holds n)
template <typename T>
__global__ void k_comb(T* z, const T* z1, const double* scal, int64_t n) {
  const double b = scal[2];
  ULOOP(i, n) z[i] = (T)((double)z1[i] + b * (double)z[i]);
}
// z += w D^-1 (r - A z1 - beta A n)
template <typename T>
__global__ void k_jcorr2(T* z, double w, const T* d, const T* r, const T* az1, const T* an, const double* scal,
                         int64_t n) {
  const double b = scal[2];
  ULOOP(i, n) z[i] = (T)((double)z[i] + w * (double)d[i] * ((double)r[i] - (double)az1[i] - b * (double)an[i]));
}
// scal[9] = G.n
__global__ __launch_bounds__(kT) void k_dot1(const double* a, const double* b, int64_t n, double* part) {
  __shared__ double sh[4];
  double x = 0.0;
  ULOOP(i, n) x += a[i] * b[i];
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
__global__ __launch_bounds__(256) void k_fin1(const double* part, int np, double* out) {
  __shared__ double sh[4];
  const double a = block_total(part, np, sh);
  if (threadIdx.x == 0) *out = a;
}
// dL/dn = beta G + (G.n / n.A n)(r1 - 2 beta A n)  (beta = n.r1 / n.A n)
__global__ void k_gbeta(double* gn, const double* G, const double* r1, const double* an, const double* scal,
                        int64_t n) {
  const double b = scal[2];
  const double c = scal[8] > 0.0 ? scal[9] / scal[8] : 0.0;
  ULOOP(i, n) gn[i] = b * G[i] + c * (r1[i] - 2.0 * b * an[i]);
}

// ------------------------------------------------------------ host side
int conv(const uint16_t* in, int cs_in, int ci, const uint16_t* wt, uint16_t* out, int cs_out, int co, int E,
         bool relu, hipStream_t s) {
  const int r = relu ? 1 : 0;
  const dim3 g((unsigned)((E + kTX - 1) / kTX), (unsigned)((E + kTY - 1) / kTY), (unsigned)((E + kTZ - 1) / kTZ));
  const int key = (co / 16) * 100 + ci;
  if (ci == 8 || ci == 16 || ci == 32 || key == 348) {
    switch (key) {
#define FL(nb, cc) \
  case nb * 100 + cc: k_conv3_flat<nb, cc><<<g, 256, 0, s>>>(in, cs_in, wt, out, cs_out, E, r); break;
      FL(1, 8) FL(1, 16) FL(1, 32) FL(2, 16) FL(2, 32) FL(3, 32) FL(5, 32) FL(3, 16) FL(3, 48)
#undef FL
      default:
        set_error("unsupported channel count");
        return CHNS_EINVAL;
    }
    CHNS_HIP(hipGetLastError());
    return CHNS_OK;
  }
  switch (co / 16) {
    case 1: k_conv3_tile<1><<<g, 256, 0, s>>>(in, cs_in, ci, wt, out, cs_out, E, r); break;
    case 2: k_conv3_tile<2><<<g, 256, 0, s>>>(in, cs_in, ci, wt, out, cs_out, E, r); break;
    case 3: k_conv3_tile<3><<<g, 256, 0, s>>>(in, cs_in, ci, wt, out, cs_out, E, r); break;
    case 4: k_conv3_tile<4><<<g, 256, 0, s>>>(in, cs_in, ci, wt, out, cs_out, E, r); break;
    case 5: k_conv3_tile<5><<<g, 256, 0, s>>>(in, cs_in, ci, wt, out, cs_out, E, r); break;
    case 7: k_conv3_tile<7><<<g, 256, 0, s>>>(in, cs_in, ci, wt, out, cs_out, E, r); break;
    default:
      set_error("unsupported channel count");
      return CHNS_EINVAL;
  }
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

int wgrad(UNet& u, int layer, const uint16_t* in, int cs_in, const uint16_t* dy, int cs_dy, int E, float scale,
          int accumulate, hipStream_t s) {
  const ULayer& l = u.L[layer];
  const int MB = (l.ci + 15) / 16, NB = l.co / 16;
  const dim3 g(kWgradSplits, 27);
#define WG(a, b) \
  k_wgrad<a, b><<<g, 64, 0, s>>>(in, cs_in, l.ci, dy, cs_dy, E, kWgradSplits, u.partial)
  const int key = MB * 10 + NB;
  switch (key) {
    case 11: WG(1, 1); break;
    case 12: WG(1, 2); break;
    case 22: WG(2, 2); break;
    case 23: WG(2, 3); break;
    case 33: WG(3, 3); break;
    case 34: WG(3, 4); break;
    case 44: WG(4, 4); break;
    case 73: WG(7, 3); break;
    case 52: WG(5, 2); break;
    case 31: WG(3, 1); break;
    default:
      set_error("unsupported weight-gradient shape");
      return CHNS_EINVAL;
  }
#undef WG
  CHNS_HIP(hipGetLastError());
  k_wgrad_reduce<<<nblk((int64_t)27 * l.ci * l.co), kT, 0, s>>>(u.partial, kWgradSplits, l.ci, l.co, MB * 16, NB * 16,
                                                                 u.grad + l.off, scale, accumulate);
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

int ensure_acts(Ctx& c, int E, bool grads, UActs** out) {
  UNet& u = *c.unet;
  for (auto& a : u.acts)
    if (a.E == E && (a.grads || !grads)) {
      *out = &a;
      return CHNS_OK;
    }
  UActs a;
  a.E = E;
  a.grads = grads;
  const int64_t V0 = (int64_t)E * E * E, V1 = V0 / 8, V2 = V1 / 8, V3 = V2 / 8;
  auto B = [&](int64_t n) { return (uint16_t*)c.dalloc(sizeof(uint16_t) * (size_t)std::max<int64_t>(n, 8)); };
  auto F = [&](int64_t n) { return (float*)c.dalloc(sizeof(float) * (size_t)std::max<int64_t>(n, 1)); };
  a.X = B(V0 * kInCh);
  a.A0 = B(V0 * 16);
  a.cat0 = B(V0 * 48);
  a.P0 = B(V1 * 16);
  a.A2 = B(V1 * 32);
  a.cat1 = B(V1 * 80);
  a.P1 = B(V2 * 32);
  a.A4 = B(V2 * 48);
  a.cat2 = B(V2 * 112);
  a.P2 = B(V3 * 48);
  a.A6 = B(V3 * 64);
  a.A7 = B(V3 * 64);
  a.A8 = B(V2 * 48);
  a.A9 = B(V2 * 48);
  a.A10 = B(V1 * 32);
  a.A11 = B(V1 * 32);
  a.A12 = B(V0 * 16);
  a.A13 = B(V0 * 16);
  a.out = F(V0);
  if (!a.X || !a.A0 || !a.cat0 || !a.P0 || !a.A2 || !a.cat1 || !a.P1 || !a.A4 || !a.cat2 || !a.P2 || !a.A6 ||
      !a.A7 || !a.A8 || !a.A9 || !a.A10 || !a.A11 || !a.A12 || !a.A13 || !a.out)
    return CHNS_ENOMEM;
  if (grads) {
    a.dA13 = B(V0 * 16);
    a.dA12 = B(V0 * 16);
    a.dcat0 = B(V0 * 48);
    a.dA11 = B(V1 * 32);
    a.dA10 = B(V1 * 32);
    a.dcat1 = B(V1 * 80);
    a.dA9 = B(V2 * 48);
    a.dA8 = B(V2 * 48);
    a.dcat2 = B(V2 * 112);
    a.dA7 = B(V3 * 64);
    a.dA6 = B(V3 * 64);
    a.dP2 = B(V3 * 48);
    a.dA4 = B(V2 * 48);
    a.dP1 = B(V2 * 32);
    a.dA2 = B(V1 * 32);
    a.dP0 = B(V1 * 16);
    a.dA0 = B(V0 * 16);
    a.target = F(V0);
    a.mask = F(V0);
    a.dout = F(V0);
    if (!a.dA13 || !a.dA12 || !a.dcat0 || !a.dA11 || !a.dA10 || !a.dcat1 || !a.dA9 || !a.dA8 || !a.dcat2 ||
        !a.dA7 || !a.dA6 || !a.dP2 || !a.dA4 || !a.dP1 || !a.dA2 || !a.dP0 || !a.dA0 || !a.target || !a.mask ||
        !a.dout)
      return CHNS_ENOMEM;
  }
  u.acts.push_back(a);
  *out = &u.acts.back();
  return CHNS_OK;
}

// forward pass on the packed input a.X
int forward(UNet& u, UActs& a, hipStream_t s) {
  const int E0 = a.E, E1 = E0 / 2, E2 = E1 / 2, E3 = E2 / 2;
  const ULayer* L = u.L;
  int rc;
#define CV(in, csi, k, out, cso, E) \
  if ((rc = conv(in, csi, L[k].ci, L[k].wf, out, cso, L[k].co, E, true, s))) return rc;
  CV(a.X, kInCh, 0, a.A0, 16, E0);
  CV(a.A0, 16, 1, a.cat0 + 32, 48, E0);
  k_pool<<<nblk((int64_t)E1 * E1 * E1 * 2), kT, 0, s>>>(a.cat0 + 32, 48, a.P0, 16, E1);
  CV(a.P0, 16, 2, a.A2, 32, E1);
  CV(a.A2, 32, 3, a.cat1 + 48, 80, E1);
  k_pool<<<nblk((int64_t)E2 * E2 * E2 * 4), kT, 0, s>>>(a.cat1 + 48, 80, a.P1, 32, E2);
  CV(a.P1, 32, 4, a.A4, 48, E2);
  CV(a.A4, 48, 5, a.cat2 + 64, 112, E2);
  k_pool<<<nblk((int64_t)E3 * E3 * E3 * 6), kT, 0, s>>>(a.cat2 + 64, 112, a.P2, 48, E3);
  CV(a.P2, 48, 6, a.A6, 64, E3);
  CV(a.A6, 64, 7, a.A7, 64, E3);
  k_up<<<nblk((int64_t)E2 * E2 * E2 * 8), kT, 0, s>>>(a.A7, 64, a.cat2, 112, E2);
  CV(a.cat2, 112, 8, a.A8, 48, E2);
  CV(a.A8, 48, 9, a.A9, 48, E2);
  k_up<<<nblk((int64_t)E1 * E1 * E1 * 6), kT, 0, s>>>(a.A9, 48, a.cat1, 80, E1);
  CV(a.cat1, 80, 10, a.A10, 32, E1);
  CV(a.A10, 32, 11, a.A11, 32, E1);
  k_up<<<nblk((int64_t)E0 * E0 * E0 * 4), kT, 0, s>>>(a.A11, 32, a.cat0, 48, E0);
  CV(a.cat0, 48, 12, a.A12, 16, E0);
  CV(a.A12, 16, 13, a.A13, 16, E0);
#undef CV
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

// backward pass from a.dout; weight gradients scaled by `scale` and added
// into u.grad when `accumulate`
int backward(UNet& u, UActs& a, float scale, int accumulate, hipStream_t s) {
  const int E0 = a.E, E1 = E0 / 2, E2 = E1 / 2, E3 = E2 / 2;
  const int64_t V0 = (int64_t)E0 * E0 * E0, V1 = V0 / 8, V2 = V1 / 8, V3 = V2 / 8;
  const ULayer* L = u.L;
  int rc;
  const unsigned gb = (unsigned)std::min<int64_t>(kRedBlocks, (V0 + kT - 1) / kT);
  k_out_bwd<<<gb, kT, 0, s>>>(a.A13, u.W + u.wout_off, a.dout, V0, a.dA13, u.gout_part);
  k_gout_reduce<<<1, 256, 0, s>>>(u.gout_part, (int)gb, u.grad + u.wout_off, scale, accumulate);
  CHNS_HIP(hipGetLastError());
  // one layer: relu mask, weight gradient, input gradient
  auto layer = [&](int k, uint16_t* dy, int cs_dy, const uint16_t* act, int cs_act, const uint16_t* in, int cs_in,
                   uint16_t* dx, int cs_dx, int E, int64_t V) -> int {
    k_relu_bwd<<<nblk(V * L[k].co / 8), kT, 0, s>>>(dy, cs_dy, act, cs_act, L[k].co, V);
    CHNS_HIP(hipGetLastError());
    int e = wgrad(u, k, in, cs_in, dy, cs_dy, E, scale, accumulate, s);
    if (e) return e;
    if (dx) return conv(dy, cs_dy, L[k].co, L[k].wb, dx, cs_dx, L[k].ci, E, false, s);
    return CHNS_OK;
  };
  if ((rc = layer(13, a.dA13, 16, a.A13, 16, a.A12, 16, a.dA12, 16, E0, V0))) return rc;
  if ((rc = layer(12, a.dA12, 16, a.A12, 16, a.cat0, 48, a.dcat0, 48, E0, V0))) return rc;
  k_up_bwd<<<nblk(V1 * 4), kT, 0, s>>>(a.dcat0, 48, a.dA11, 32, E1);
  if ((rc = layer(11, a.dA11, 32, a.A11, 32, a.A10, 32, a.dA10, 32, E1, V1))) return rc;
  if ((rc = layer(10, a.dA10, 32, a.A10, 32, a.cat1, 80, a.dcat1, 80, E1, V1))) return rc;
  k_up_bwd<<<nblk(V2 * 6), kT, 0, s>>>(a.dcat1, 80, a.dA9, 48, E2);
  if ((rc = layer(9, a.dA9, 48, a.A9, 48, a.A8, 48, a.dA8, 48, E2, V2))) return rc;
  if ((rc = layer(8, a.dA8, 48, a.A8, 48, a.cat2, 112, a.dcat2, 112, E2, V2))) return rc;
  k_up_bwd<<<nblk(V3 * 8), kT, 0, s>>>(a.dcat2, 112, a.dA7, 64, E3);
  if ((rc = layer(7, a.dA7, 64, a.A7, 64, a.A6, 64, a.dA6, 64, E3, V3))) return rc;
  if ((rc = layer(6, a.dA6, 64, a.A6, 64, a.P2, 48, a.dP2, 48, E3, V3))) return rc;
  k_pool_bwd_add<<<nblk(V2 * 6), kT, 0, s>>>(a.dP2, 48, a.dcat2 + 64, 112, E2);
  if ((rc = layer(5, a.dcat2 + 64, 112, a.cat2 + 64, 112, a.A4, 48, a.dA4, 48, E2, V2))) return rc;
  if ((rc = layer(4, a.dA4, 48, a.A4, 48, a.P1, 32, a.dP1, 32, E2, V2))) return rc;
  k_pool_bwd_add<<<nblk(V1 * 4), kT, 0, s>>>(a.dP1, 32, a.dcat1 + 48, 80, E1);
  if ((rc = layer(3, a.dcat1 + 48, 80, a.cat1 + 48, 80, a.A2, 32, a.dA2, 32, E1, V1))) return rc;
  if ((rc = layer(2, a.dA2, 32, a.A2, 32, a.P0, 16, a.dP0, 16, E1, V1))) return rc;
  k_pool_bwd_add<<<nblk(V0 * 2), kT, 0, s>>>(a.dP0, 16, a.dcat0 + 32, 48, E0);
  if ((rc = layer(1, a.dcat0 + 32, 48, a.cat0 + 32, 48, a.A0, 16, a.dA0, 16, E0, V0))) return rc;
  if ((rc = layer(0, a.dA0, 16, a.A0, 16, a.X, kInCh, nullptr, 0, E0, V0))) return rc;
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

int prep_weights(UNet& u, hipStream_t s) {
  for (int k = 0; k < kLayers; ++k) {
    const ULayer& l = u.L[k];
    k_prep_weights<<<nblk((int64_t)27 * l.ci * l.co), kT, 0, s>>>(u.W + l.off, l.ci, l.co, l.wf, l.wb);
  }
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

double lratio(const Ctx& c) {
  const double r = c.prm.rho_plus / c.prm.rho_minus;
  return r > 1.0 ? std::log(r) : 1.0;
}

// rho(phi) = alpha phi* + beta, normalised by rho+
void rho_ab(const Ctx& c, double* a, double* b) {
  *a = (c.prm.rho_plus - c.prm.rho_minus) / (2.0 * c.prm.rho_plus);
  *b = (c.prm.rho_plus + c.prm.rho_minus) / (2.0 * c.prm.rho_plus);
}

int check_grid(const Ctx& c) {
  if (c.dm.dim != 3 || !c.dm.structured) {
    set_error("training and crop passes of the network need a uniform 3D mesh");
    return CHNS_EINVAL;
  }
  return CHNS_OK;
}

// The preconditioner runs on uniform 3D meshes directly and on 3D octrees of
// the whole cube refined to at least the grid level through the grid.
int check_pc(const Ctx& c) {
  if (c.dm.dim == 3 && c.dm.structured) return CHNS_OK;
  if (c.dm.dim != 3 || !c.host || c.host->carve_level != 0 || c.host->max_level < kGridLevel) {
    set_error("the learned preconditioner needs a 3D octree of the whole cube with max_level >= " +
              std::to_string(kGridLevel));
    return CHNS_EINVAL;
  }
  return CHNS_OK;
}
// nodes per axis - 1 of the grid the network sees
int net_side(const Ctx& c) { return c.dm.structured ? c.dm.side : (1 << kGridLevel); }

// splitmix64 -> two uniforms -> Box-Muller normal
uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double normal(uint64_t& s) {
  const double u1 = ((splitmix(s) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  const double u2 = (splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

}  // namespace

// ---------------------------------------------------------------- API
int unet_create(Ctx& c) {
  if (c.unet) return CHNS_OK;
  c.unet = new UNet();
  UNet& u = *c.unet;
  const int c0 = kCh[0], c1 = kCh[1], c2 = kCh[2], c3 = kCh[3];
  const int shapes[kLayers][2] = {{kInCh, c0}, {c0, c0}, {c0, c1}, {c1, c1}, {c1, c2}, {c2, c2}, {c2, c3},
                                  {c3, c3}, {c3 + c2, c2}, {c2, c2}, {c2 + c1, c1}, {c1, c1}, {c1 + c0, c0},
                                  {c0, c0}};
  size_t off = 0, nbf = 0;
  for (int k = 0; k < kLayers; ++k) {
    u.L[k].ci = shapes[k][0];
    u.L[k].co = shapes[k][1];
    u.L[k].off = off;
    off += (size_t)27 * shapes[k][0] * shapes[k][1];
  }
  u.wout_off = off;
  u.nparam = off + 16;
  nbf = 2 * off;
  u.W = (float*)c.dalloc(sizeof(float) * u.nparam);
  u.m = (float*)c.dalloc(sizeof(float) * u.nparam);
  u.v = (float*)c.dalloc(sizeof(float) * u.nparam);
  u.grad = (float*)c.dalloc(sizeof(float) * u.nparam);
  u.wbf = (uint16_t*)c.dalloc(sizeof(uint16_t) * nbf);
  size_t pmax = 0;
  for (int k = 0; k < kLayers; ++k)
    pmax = std::max(pmax, (size_t)kWgradSplits * 27 * ((u.L[k].ci + 15) / 16 * 16) * u.L[k].co);
  u.partial = (float*)c.dalloc(sizeof(float) * pmax);
  u.partial_cap = pmax;
  u.red = (double*)c.dalloc(sizeof(double) * 3 * kRedBlocks);  // up to three partial rows
  u.scal = (double*)c.dalloc(sizeof(double) * 16);
  u.gout_part = (float*)c.dalloc(sizeof(float) * 16 * kRedBlocks);
  if (!u.W || !u.m || !u.v || !u.grad || !u.wbf || !u.partial || !u.red || !u.scal || !u.gout_part)
    return CHNS_ENOMEM;
  CHNS_HIP(hipHostMalloc((void**)&u.scal_host, sizeof(double) * 16, hipHostMallocDefault));
  size_t b = 0;
  for (int k = 0; k < kLayers; ++k) {
    const size_t n = (size_t)27 * u.L[k].ci * u.L[k].co;
    u.L[k].wf = u.wbf + b;
    u.L[k].wb = u.wbf + b + n;
    b += 2 * n;
  }
  return CHNS_OK;
}

void unet_destroy(Ctx& c) {
  if (!c.unet) return;
  if (c.unet->scal_host) (void)hipHostFree(c.unet->scal_host);
  delete c.unet;
  c.unet = nullptr;
}

static int set_params(Ctx& c, const std::vector<float>& w, float K, float omega, hipStream_t s) {
  UNet& u = *c.unet;
  CHNS_HIP(hipMemcpyAsync(u.W, w.data(), sizeof(float) * u.nparam, hipMemcpyHostToDevice, s));
  CHNS_HIP(hipMemsetAsync(u.m, 0, sizeof(float) * u.nparam, s));
  CHNS_HIP(hipMemsetAsync(u.v, 0, sizeof(float) * u.nparam, s));
  CHNS_HIP(hipMemsetAsync(u.grad, 0, sizeof(float) * u.nparam, s));
  int rc = prep_weights(u, s);
  if (rc) return rc;
  CHNS_HIP(hipStreamSynchronize(s));
  u.K = K;
  u.omega = omega;
  u.step = 0;
  u.ready = true;
  return CHNS_OK;
}

int unet_init(Ctx& c, uint64_t seed, float K, float omega, hipStream_t s) {
  int rc = unet_create(c);
  if (rc) return rc;
  UNet& u = *c.unet;
  std::vector<float> w(u.nparam);
  uint64_t st = seed;
  for (int k = 0; k < kLayers; ++k) {
    // He initialisation over the fan-in of the real input channels
    const int fan = 27 * (k == 0 ? 2 : u.L[k].ci);
    const double sd = std::sqrt(2.0 / fan);
    for (int t = 0; t < 27; ++t)
      for (int i = 0; i < u.L[k].ci; ++i)
        for (int o = 0; o < u.L[k].co; ++o) {
          const double x = normal(st) * sd;
          w[u.L[k].off + ((size_t)t * u.L[k].ci + i) * u.L[k].co + o] = (k == 0 && i >= 2) ? 0.0f : (float)x;
        }
  }
  for (int c2 = 0; c2 < 16; ++c2) w[u.wout_off + c2] = (float)(normal(st) * std::sqrt(1.0 / 16));
  return set_params(c, w, K, omega, s);
}

// blob: "CHNSUNET", u32 version (1 or 2), u32 layers, f32 K, [version 2:
// f32 omega], per layer u32 ci, u32 co, f32 W[27][ci][co]; u32 16,
// f32 w_out[16]
int unet_load(Ctx& c, const void* blob, size_t n, hipStream_t s) {
  int rc = unet_create(c);
  if (rc) return rc;
  UNet& u = *c.unet;
  const uint8_t* p = (const uint8_t*)blob;
  size_t pos = 0;
  auto take = [&](void* dst, size_t k) -> bool {
    if (pos + k > n) return false;
    std::memcpy(dst, p + pos, k);
    pos += k;
    return true;
  };
  char magic[8];
  uint32_t ver = 0, nl = 0;
  float K = 1.0f, omega = 0.0f;
  if (!blob || !take(magic, 8) || std::memcmp(magic, "CHNSUNET", 8) != 0 || !take(&ver, 4) ||
      (ver != 1 && ver != 2) || !take(&nl, 4) || nl != kLayers || !take(&K, 4) || (ver == 2 && !take(&omega, 4)) ||
      !(K >= 0.0f) || !(omega >= 0.0f && omega < 2.0f)) {
    set_error("not a U-Net weight blob of this library");
    return CHNS_EINVAL;
  }
  std::vector<float> w(u.nparam);
  for (int k = 0; k < kLayers; ++k) {
    uint32_t ci = 0, co = 0;
    if (!take(&ci, 4) || !take(&co, 4) || (int)ci != u.L[k].ci || (int)co != u.L[k].co ||
        !take(w.data() + u.L[k].off, sizeof(float) * 27 * ci * co)) {
      set_error("U-Net blob does not match the network shape");
      return CHNS_EINVAL;
    }
  }
  uint32_t no = 0;
  if (!take(&no, 4) || no != 16 || !take(w.data() + u.wout_off, sizeof(float) * 16) || pos != n) {
    set_error("U-Net blob is truncated or has trailing bytes");
    return CHNS_EINVAL;
  }
  return set_params(c, w, K, omega, s);
}

size_t unet_blob_size(const Ctx& c) {
  if (!c.unet) return 0;
  const UNet& u = *c.unet;
  return 8 + 4 + 4 + 4 + 4 + kLayers * 8 + (u.nparam - 16) * 4 + 4 + 64;
}

int unet_save(Ctx& c, void* blob, size_t cap, size_t* n) {
  if (!c.unet || !c.unet->ready) {
    set_error("no U-Net weights in this context");
    return CHNS_ESTATE;
  }
  UNet& u = *c.unet;
  const size_t need = unet_blob_size(c);
  *n = need;
  if (!blob) return CHNS_OK;
  if (cap < need) {
    set_error("blob buffer too small");
    return CHNS_EINVAL;
  }
  std::vector<float> w(u.nparam);
  CHNS_HIP(hipMemcpy(w.data(), u.W, sizeof(float) * u.nparam, hipMemcpyDeviceToHost));
  uint8_t* p = (uint8_t*)blob;
  size_t pos = 0;
  auto put = [&](const void* src, size_t k) {
    std::memcpy(p + pos, src, k);
    pos += k;
  };
  const uint32_t ver = 2, nl = kLayers, no = 16;
  put("CHNSUNET", 8);
  put(&ver, 4);
  put(&nl, 4);
  put(&u.K, 4);
  put(&u.omega, 4);
  for (int k = 0; k < kLayers; ++k) {
    const uint32_t ci = u.L[k].ci, co = u.L[k].co;
    put(&ci, 4);
    put(&co, 4);
    put(w.data() + u.L[k].off, sizeof(float) * 27 * ci * co);
  }
  put(&no, 4);
  put(w.data() + u.wout_off, sizeof(float) * 16);
  return CHNS_OK;
}

int unet_gradients(Ctx& c, float* host, size_t n) {
  if (!c.unet || !c.unet->ready) {
    set_error("no U-Net weights in this context");
    return CHNS_ESTATE;
  }
  if (n != c.unet->nparam) {
    set_error("gradient buffer must hold exactly the parameter count");
    return CHNS_EINVAL;
  }
  CHNS_HIP(hipMemcpy(host, c.unet->grad, sizeof(float) * n, hipMemcpyDeviceToHost));
  return CHNS_OK;
}

size_t unet_param_count(const Ctx& c) { return c.unet ? c.unet->nparam : 0; }

static int pack_sample(Ctx& c, UActs& a, const double* phi, const double* r, const double* e, const int32_t* origin,
                       int flip, hipStream_t s) {
  UNet& u = *c.unet;
  const int64_t n = c.dm.n;
  const unsigned g = (unsigned)std::min<int64_t>(kRedBlocks, (n + kT - 1) / kT);
  k_sumsq<double><<<g, kT, 0, s>>>(r, n, u.red);
  k_rms<<<1, 256, 0, s>>>(u.red, (int)g, n, u.scal);
  PackGeo geo{c.dm.side, a.E, origin ? origin[0] : 0, origin ? origin[1] : 0, origin ? origin[2] : 0, flip};
  double al, be;
  rho_ab(c, &al, &be);
  const int64_t V = (int64_t)a.E * a.E * a.E;
  k_pack<double><<<nblk(V), kT, 0, s>>>(geo, phi, r, e, u.scal, al, be, 1.0 / lratio(c), u.K, a.X, a.target,
                                        a.mask);
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

int unet_forward_crop(Ctx& c, const double* phi, const double* r, const int32_t* origin, int flip, int crop,
                      float* out, hipStream_t s) {
  int rc;
  if ((rc = check_grid(c))) return rc;
  if (!c.unet || !c.unet->ready) {
    set_error("no U-Net weights in this context");
    return CHNS_ESTATE;
  }
  if (crop < 8 || crop % 8) {
    set_error("crop edge must be a positive multiple of 8");
    return CHNS_EINVAL;
  }
  for (int k = 0; k < 3; ++k)
    if (origin && (origin[k] < 0 || origin[k] > c.dm.side)) {
      set_error("crop origin outside the node grid");
      return CHNS_EINVAL;
    }
  UActs* a = nullptr;
  if ((rc = ensure_acts(c, crop, false, &a))) return rc;
  if ((rc = pack_sample(c, *a, phi, r, nullptr, origin, flip, s))) return rc;
  if ((rc = forward(*c.unet, *a, s))) return rc;
  const int64_t V = (int64_t)crop * crop * crop;
  k_out<<<nblk(V), kT, 0, s>>>(a->A13, c.unet->W + c.unet->wout_off, out, V);
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

static int adam_update(UNet& u, float lr, hipStream_t s) {
  u.step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, u.step)), c2 = (float)(1.0 - std::pow(b2, u.step));
  k_adam<<<nblk((int64_t)u.nparam), kT, 0, s>>>(u.W, u.m, u.v, u.grad, (int64_t)u.nparam, lr, (float)b1, (float)b2,
                                                c1, c2, 1e-8f);
  CHNS_HIP(hipGetLastError());
  return prep_weights(u, s);
}

// network part of the preconditioner on a node vector x: rms(x) -> scal[0],
// pack, forward, z = rms(x) K Net (no projection)
template <typename T>
static int net_nodes(Ctx& c, UActs& a, int side, int64_t n, const double* phi, const T* x, T* z, hipStream_t s) {
  UNet& u = *c.unet;
  const unsigned g = (unsigned)std::min<int64_t>(kRedBlocks, (n + kT - 1) / kT);
  const PackGeo geo{side, a.E, 0, 0, 0, 0};
  double al, be;
  rho_ab(c, &al, &be);
  const int64_t V = (int64_t)a.E * a.E * a.E;
  k_sumsq<T><<<g, kT, 0, s>>>(x, n, u.red);
  k_rms<<<1, 256, 0, s>>>(u.red, (int)g, n, u.scal);
  k_pack<T><<<nblk(V), kT, 0, s>>>(geo, phi, x, nullptr, u.scal, al, be, 1.0 / lratio(c), u.K, a.X, nullptr,
                                   nullptr);
  CHNS_HIP(hipGetLastError());
  int rc = forward(u, a, s);
  if (rc) return rc;
  k_unpack<T><<<nblk(V), kT, 0, s>>>(geo, a.A13, u.W + u.wout_off, u.scal, u.K, z);
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

// network part of the preconditioner on a mesh vector: on a uniform mesh
// the node grid is the mesh's own; otherwise z = P Net(R x) on the grid
// (phi~ sampled there by Q when the solve is prepared)
template <typename T>
static int net_apply(Ctx& c, UActs& a, const T* x, T* z, hipStream_t s) {
  if (c.dm.structured) return net_nodes<T>(c, a, c.dm.side, c.dm.n, c.phi64, x, z, s);
  UNet& u = *c.unet;
  constexpr bool f64 = sizeof(T) == 8;
  T* xg = f64 ? (T*)u.xg64[0] : (T*)u.xg32[0];
  T* zg = f64 ? (T*)u.xg64[1] : (T*)u.xg32[1];
  if (!u.grid_built || !xg || !zg) {
    set_error("grid transfers of the learned preconditioner are not prepared");
    return CHNS_ESTATE;
  }
  k_csr_apply<T><<<nblk(u.n_grid), kT, 0, s>>>(u.gR_ptr, u.gR_col, u.gR_val, x, xg, u.n_grid);
  CHNS_HIP(hipGetLastError());
  int rc = net_nodes<T>(c, a, 1 << kGridLevel, u.n_grid, u.phig, xg, zg, s);
  if (rc) return rc;
  k_csr_apply<T><<<nblk(c.dm.n), kT, 0, s>>>(u.gP_ptr, u.gP_col, u.gP_val, zg, z, c.dm.n);
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

// Full-grid A-norm objective: L = (e - z)^T A (e - z) / e^T r for the
// preconditioner output z (A e = r), i.e. (z^T A z - 2 z^T r + e^T r) / e^T r,
// G0 = dL/dz = 2 (A z - r) / e^T r.  With smoothing
// z = (I - w D^-1 A) z2 + w D^-1 r, z2 = z1 + beta n, so G = dL/dz2 =
// (I - w A D^-1) G0, and through beta = n.r1 / n.A n:
// dL/dn = beta G + (G.n / n.A n)(r1 - 2 beta A n).  The context's phase field
// is set to each sample's.
static int train_energy(Ctx& c, const chns_pc_batch& b, float lr, float* loss, hipStream_t s) {
  UNet& u = *c.unet;
  const int64_t n = c.dm.n;
  int rc;
  if (!u.zb) {
    u.zb = (double*)c.dalloc(sizeof(double) * n);
    u.qb = (double*)c.dalloc(sizeof(double) * n);
    for (auto& t : u.tb) t = (double*)c.dalloc(sizeof(double) * n);
    for (auto t : u.tb)
      if (!t) return CHNS_ENOMEM;
    if (!u.zb || !u.qb) return CHNS_ENOMEM;
  }
  const int E = ((c.dm.side + 1 + 7) / 8) * 8;
  UActs* a = nullptr;
  if ((rc = ensure_acts(c, E, true, &a))) return rc;
  const int64_t V = (int64_t)E * E * E;
  const unsigned g = (unsigned)std::min<int64_t>(kRedBlocks, (n + kT - 1) / kT);
  const unsigned gn = nblk(n);
  const PackGeo geo{c.dm.side, E, 0, 0, 0, 0};
  const double w = u.omega;
  double *d = u.tb[0], *z1 = u.tb[1], *az1 = u.tb[2], *r1 = u.tb[3], *an = u.tb[4], *G = u.tb[5], *h = u.tb[6],
         *ah = u.tb[7], *gnet = u.tb[8], *z = u.tb[9];
  double* net = u.zb;
  double total = 0.0;
  ApplyOut plain{};
  for (int k = 0; k < b.n; ++k) {
    if (!b.phi[k] || !b.r[k] || !b.e[k]) {
      set_error("null field in training batch");
      return CHNS_EINVAL;
    }
    const double* r = b.r[k];
    if ((rc = launch_set_phase(c, b.phi[k], nullptr, s))) return rc;
    const double* xin = r;
    if (w > 0.0) {
      if ((rc = launch_diagonal(c, CHNS_OP_PRESSURE, CHNS_FP64, d, true, s))) return rc;
      k_wdinv<double><<<gn, kT, 0, s>>>(z1, w, d, r, n);
      if ((rc = launch_apply(c, CHNS_OP_PRESSURE, CHNS_FP64, z1, az1, s, plain))) return rc;
      k_diffv<double><<<gn, kT, 0, s>>>(r1, r, az1, n);
      CHNS_HIP(hipGetLastError());
      xin = r1;
    }
    if ((rc = net_nodes<double>(c, *a, c.dm.side, c.dm.n, b.phi[k], xin, net, s))) return rc;
    const double* zz = net;
    if (w > 0.0) {
      if ((rc = launch_apply(c, CHNS_OP_PRESSURE, CHNS_FP64, net, an, s, plain))) return rc;
      k_dot2<double><<<g, kT, 0, s>>>(net, r1, an, n, u.red);
      k_beta<<<1, 256, 0, s>>>(u.red, (int)g, u.scal);
      CHNS_HIP(hipMemcpyAsync(z, net, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      k_comb<double><<<gn, kT, 0, s>>>(z, z1, u.scal, n);
      k_jcorr2<double><<<gn, kT, 0, s>>>(z, w, d, r, az1, an, u.scal, n);
      CHNS_HIP(hipGetLastError());
      zz = z;
    }
    if ((rc = launch_apply(c, CHNS_OP_PRESSURE, CHNS_FP64, zz, u.qb, s, plain))) return rc;
    k_dot3<<<g, kT, 0, s>>>(zz, u.qb, r, b.e[k], n, u.red);
    k_fin3<<<1, 256, 0, s>>>(u.red, (int)g, u.scal);
    k_grad_anorm<<<gn, kT, 0, s>>>(u.qb, r, u.scal, G, n);
    CHNS_HIP(hipGetLastError());
    const double* gout = G;
    if (w > 0.0) {
      k_wdinv<double><<<gn, kT, 0, s>>>(h, 1.0, d, G, n);
      if ((rc = launch_apply(c, CHNS_OP_PRESSURE, CHNS_FP64, h, ah, s, plain))) return rc;
      k_axpy_neg<<<gn, kT, 0, s>>>(G, w, ah, n);
      k_dot1<<<g, kT, 0, s>>>(G, net, n, u.red);
      k_fin1<<<1, 256, 0, s>>>(u.red, (int)g, u.scal + 9);
      k_gbeta<<<gn, kT, 0, s>>>(gnet, G, r1, an, u.scal, n);
      CHNS_HIP(hipGetLastError());
      gout = gnet;
    }
    k_dout_nodes<<<nblk(V), kT, 0, s>>>(geo, gout, u.scal, u.K, a->dout);
    CHNS_HIP(hipGetLastError());
    if ((rc = backward(u, *a, 1.0f / (float)b.n, k > 0 ? 1 : 0, s))) return rc;
    CHNS_HIP(hipMemcpyAsync(u.scal_host, u.scal, sizeof(double) * 16, hipMemcpyDeviceToHost, s));
    CHNS_HIP(hipStreamSynchronize(s));
    total += u.scal_host[7];
  }
  if (loss) *loss = (float)(total / b.n);
  if (lr > 0.0f && (rc = adam_update(u, lr, s))) return rc;
  CHNS_HIP(hipStreamSynchronize(s));
  return CHNS_OK;
}

int unet_train_step(Ctx& c, const chns_pc_batch& b, float lr, float* loss, hipStream_t s) {
  int rc;
  if ((rc = check_grid(c))) return rc;
  if (!c.unet || !c.unet->ready) {
    set_error("no U-Net weights in this context");
    return CHNS_ESTATE;
  }
  if (!(c.unet->K > 0.0f)) {
    set_error("training needs a positive output scale K");
    return CHNS_EINVAL;
  }
  if (b.objective == CHNS_PC_OBJ_ANORM) {
    if (b.n < 1 || !b.phi || !b.r || !b.e) {
      set_error("bad training batch");
      return CHNS_EINVAL;
    }
    return train_energy(c, b, lr, loss, s);
  }
  if (b.objective != CHNS_PC_OBJ_CROP_MSE) {
    set_error("unknown training objective");
    return CHNS_EINVAL;
  }
  if (b.n < 1 || !b.phi || !b.r || !b.e || !b.origin || b.crop < 8 || b.crop % 8) {
    set_error("bad training batch");
    return CHNS_EINVAL;
  }
  for (int k = 0; k < 3 * b.n; ++k)
    if (b.origin[k] < 0 || b.origin[k] > c.dm.side) {
      set_error("crop origin outside the node grid");
      return CHNS_EINVAL;
    }
  UNet& u = *c.unet;
  UActs* a = nullptr;
  if ((rc = ensure_acts(c, b.crop, true, &a))) return rc;
  const int64_t V = (int64_t)b.crop * b.crop * b.crop;
  const unsigned gl = (unsigned)std::min<int64_t>(kRedBlocks, (V + kT - 1) / kT);
  double total = 0.0;
  const float scale = 1.0f / (float)b.n;
  for (int k = 0; k < b.n; ++k) {
    if (!b.phi[k] || !b.r[k] || !b.e[k]) {
      set_error("null field in training batch");
      return CHNS_EINVAL;
    }
    if ((rc = pack_sample(c, *a, b.phi[k], b.r[k], b.e[k], b.origin + 3 * k, b.flip ? b.flip[k] : 0, s))) return rc;
    if ((rc = forward(u, *a, s))) return rc;
    k_out<<<nblk(V), kT, 0, s>>>(a->A13, u.W + u.wout_off, a->out, V);
    k_mse<<<gl, kT, 0, s>>>(a->out, a->target, a->mask, V, u.red);
    k_sum2<<<1, 256, 0, s>>>(u.red, (int)gl, u.scal + 2);
    k_dout<<<nblk(V), kT, 0, s>>>(a->out, a->target, a->mask, u.scal + 2, a->dout, V);
    CHNS_HIP(hipGetLastError());
    if ((rc = backward(u, *a, scale, k > 0 ? 1 : 0, s))) return rc;
    CHNS_HIP(hipMemcpyAsync(u.scal_host, u.scal, sizeof(double) * 4, hipMemcpyDeviceToHost, s));
    CHNS_HIP(hipStreamSynchronize(s));
    total += u.scal_host[3] > 0.0 ? u.scal_host[2] / u.scal_host[3] : 0.0;
  }
  if (loss) *loss = (float)(total / b.n);
  if (lr > 0.0f && (rc = adam_update(u, lr, s))) return rc;
  CHNS_HIP(hipStreamSynchronize(s));
  return CHNS_OK;
}

bool unet_ready(const Ctx& c) { return c.unet && c.unet->ready; }

// activations of the network's grid and the smoothing work vectors,
// allocated before any graph capture; on adaptive meshes the grid transfers
// (built on the host once per context) and phi~ at the grid points
int unet_prepare(Ctx& c, hipStream_t s) {
  int rc;
  if ((rc = check_pc(c))) return rc;
  UNet& u = *c.unet;
  for (int k = 0; k < 4; ++k) {
    if (!u.hb64[k]) u.hb64[k] = (double*)c.dalloc(sizeof(double) * c.dm.n);
    if (!u.hb32[k]) u.hb32[k] = (float*)c.dalloc(sizeof(float) * c.dm.n);
    if (!u.hb64[k] || !u.hb32[k]) return CHNS_ENOMEM;
  }
  if (!c.dm.structured) {
    if (!u.grid_built) {
      GridTransfer t;
      std::string msg;
      if ((rc = build_grid_transfer(*c.host, kGridLevel, t, msg))) {
        set_error(msg);
        return rc;
      }
      u.n_grid = (int64_t)t.R_ptr.size() - 1;
      auto up = [&](auto** dst, const auto& v) -> int {
        using E = typename std::decay_t<decltype(v)>::value_type;
        *dst = (E*)c.dalloc(sizeof(E) * std::max<size_t>(v.size(), 1));
        if (!*dst) return CHNS_ENOMEM;
        if (!v.empty()) CHNS_HIP(hipMemcpy(*dst, v.data(), sizeof(E) * v.size(), hipMemcpyHostToDevice));
        return CHNS_OK;
      };
      if ((rc = up(&u.gP_ptr, t.P_ptr)) || (rc = up(&u.gP_col, t.P_col)) || (rc = up(&u.gP_val, t.P_val)) ||
          (rc = up(&u.gR_ptr, t.R_ptr)) || (rc = up(&u.gR_col, t.R_col)) || (rc = up(&u.gR_val, t.R_val)) ||
          (rc = up(&u.gQ_ptr, t.Q_ptr)) || (rc = up(&u.gQ_col, t.Q_col)) || (rc = up(&u.gQ_val, t.Q_val)))
        return rc;
      u.phig = (double*)c.dalloc(sizeof(double) * u.n_grid);
      for (int k = 0; k < 2; ++k) {
        u.xg64[k] = (double*)c.dalloc(sizeof(double) * u.n_grid);
        u.xg32[k] = (float*)c.dalloc(sizeof(float) * u.n_grid);
        if (!u.xg64[k] || !u.xg32[k]) return CHNS_ENOMEM;
      }
      if (!u.phig) return CHNS_ENOMEM;
      u.grid_built = true;
    }
    k_csr_apply<double><<<nblk(u.n_grid), kT, 0, s>>>(u.gQ_ptr, u.gQ_col, u.gQ_val, c.phi64, u.phig, u.n_grid);
    CHNS_HIP(hipGetLastError());
  }
  UActs* a = nullptr;
  return ensure_acts(c, ((net_side(c) + 1 + 7) / 8) * 8, false, &a);
}

// Preconditioner (kernels only, graph-capturable; the phase field is the
// context's phi~ and D^-1 its exact inverse diagonal).  Network alone:
// z = N(r); with smoothing: z1 = w D^-1 r, r1 = r - A z1, n = N(r1),
// z2 = z1 + beta n (beta = n.r1 / n.A n), z = z2 + w D^-1 (r - A z1 - beta A n).
// Then 1^T z = 0.
template <typename T>
int unet_apply(Ctx& c, const T* r, T* z, hipStream_t s) {
  int rc;
  if ((rc = check_pc(c))) return rc;
  UNet& u = *c.unet;
  const int E = ((net_side(c) + 1 + 7) / 8) * 8;
  UActs* a = nullptr;
  if ((rc = ensure_acts(c, E, false, &a))) return rc;
  const int64_t n = c.dm.n;
  const unsigned g = (unsigned)std::min<int64_t>(kRedBlocks, (n + kT - 1) / kT);
  const unsigned gn = nblk(n);
  const double w = u.omega;
  if (w > 0.0) {
    constexpr bool f64 = sizeof(T) == 8;
    T* const* hb = f64 ? (T* const*)u.hb64 : (T* const*)u.hb32;
    T *z1 = hb[0], *az1 = hb[1], *r1 = hb[2], *an = hb[3];
    const T* d = f64 ? (const T*)c.diag64 : (const T*)c.diag32;
    const int prec = f64 ? CHNS_FP64 : CHNS_FP32;
    if (!z1 || !az1 || !r1 || !an || !d || !c.diag_valid) {
      set_error("preconditioner work buffers or diagonal missing");
      return CHNS_ESTATE;
    }
    ApplyOut plain{};
    k_wdinv<T><<<gn, kT, 0, s>>>(z1, w, d, r, n);
    if ((rc = launch_apply(c, CHNS_OP_PRESSURE, prec, z1, az1, s, plain))) return rc;
    k_diffv<T><<<gn, kT, 0, s>>>(r1, r, az1, n);
    CHNS_HIP(hipGetLastError());
    if ((rc = net_apply<T>(c, *a, r1, z, s))) return rc;
    if ((rc = launch_apply(c, CHNS_OP_PRESSURE, prec, z, an, s, plain))) return rc;
    k_dot2<T><<<g, kT, 0, s>>>(z, r1, an, n, u.red);
    k_beta<<<1, 256, 0, s>>>(u.red, (int)g, u.scal);
    k_comb<T><<<gn, kT, 0, s>>>(z, z1, u.scal, n);
    k_jcorr2<T><<<gn, kT, 0, s>>>(z, w, d, r, az1, an, u.scal, n);
    CHNS_HIP(hipGetLastError());
  } else if ((rc = net_apply<T>(c, *a, r, z, s))) {
    return rc;
  }
  k_sum_part<T><<<g, kT, 0, s>>>(z, n, u.red);
  k_mean<<<1, 256, 0, s>>>(u.red, (int)g, n, u.scal);
  k_sub<T><<<gn, kT, 0, s>>>(z, n, u.scal);
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}
template int unet_apply<double>(Ctx&, const double*, double*, hipStream_t);
template int unet_apply<float>(Ctx&, const float*, float*, hipStream_t);

}  // namespace chns
