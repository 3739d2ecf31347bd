// Matrix-free Q1 operator applies on bricks of octree leaves (gfx950).
//
// y = P^T (sum_e K_e) P x without assembling anything:
//   * a brick is an aligned cube of B^d leaves of one level; one wavefront
//     owns 64/B^(d-1) bricks and walks them layer by layer along the last
//     axis, one leaf column per lane;
//   * each node layer of a brick is gathered once into LDS through the
//     brick's node table; hanging entries are interpolated from their parents
//     on the fly (the constraint P, paper Sec. 4.3 and Fig. 1 caption);
//   * every lane evaluates its leaf with sum-factorised 2-point Gauss
//     quadrature (the element operators below);
//   * leaf results are summed per node in LDS in a fixed order; nodes inside
//     a brick are written straight to y, nodes on a brick face go to a slot
//     buffer, and a second pass (k_combine) adds the slots of every shared
//     node in a fixed order, applying P^T for hanging entries.  No atomics:
//     the result is bitwise reproducible.
#include "brick_geom.h"
#include "chns_internal.h"

namespace chns {
namespace {

constexpr double kGauss = 0.57735026918962576451;  // 1/sqrt(3)

// ------------------------------------------------------------ arithmetic
__device__ __forceinline__ double rcp_t(double r) {
  // hardware estimate refined by two Newton steps (error well below 1e-15)
  double y = __builtin_amdgcn_rcp(r);
  double e = __builtin_fma(-r, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-r, y, 1.0);
  return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float rcp_t(float r) { return __builtin_amdgcn_rcpf(r); }
// Pull back of the (scaled) phase field to its physical range.  FP64 fields
// hold phi in [-lim, lim]; FP32 fields hold 1 + phi in [0, 2 lim].
__device__ __forceinline__ double clamp_t(double v, double lim) { return fmin(fmax(v, -lim), lim); }
__device__ __forceinline__ float clamp_t(float v, float lim) { return __builtin_amdgcn_fmed3f(v, 0.0f, 2.0f * lim); }

// 1D two-node / two-Gauss-point transform, scaled by 2: (a, b) nodal values
// -> values at xi = -1/sqrt3, +1/sqrt3.  The 2x2 matrix is symmetric, so the
// same transform also applies the transpose.
template <typename T>
__device__ __forceinline__ void pair_tf(T& a, T& b) {
  T t = a + b;
  T u = b - a;
  a = __builtin_fma(T(-kGauss), u, t);
  b = __builtin_fma(T(kGauss), u, t);
}
template <int N, int BIT, typename T>
__device__ __forceinline__ void stage(T* v) {
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (!(i & BIT)) pair_tf(v[i], v[i | BIT]);
}
template <int DIM, typename T>
__device__ __forceinline__ void all_stages(T* v) {
  constexpr int N = 1 << DIM;
  stage<N, 1>(v);
  stage<N, 2>(v);
  if constexpr (DIM == 3) stage<N, 4>(v);
}
__host__ __device__ constexpr int insert0(int r, int d) { return (r & ((1 << d) - 1)) | ((r >> d) << (d + 1)); }

// --------------------------------------------------------- element operators
// Folded constants: with values scaled by 2^d through the stages, the Gauss
// weights (1), det J = (h/2)^d and the (2/h)^2 of two gradients collapse into
// per-level powers of two (exact), so c_q = 1/rho(phi*_q) costs one fma, one
// clamp and one reciprocal per Gauss point.

// Pressure Poisson: y_a = sum_q detJ (2/h)^2 c_q gradN_a . grad x,
// c_q = 1/rho(clamp(phi_q)) (Def. 2, VMS pressure Poisson; pull back remark).
template <int DIM, typename T>
__device__ __forceinline__ void elem_pp(const T* x, const T* ph, T A, T Bc, T* y) {
  constexpr int NC = 1 << DIM, H = NC / 2;
  T q[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) q[i] = ph[i];
  all_stages<DIM>(q);
  T c[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) c[i] = rcp_t(__builtin_fma(A, clamp_t(q[i], T(NC)), Bc));
#pragma unroll
  for (int i = 0; i < NC; ++i) y[i] = T(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    T g[H];
#pragma unroll
    for (int r = 0; r < H; ++r) {
      const int lo = insert0(r, d), hi = lo | (1 << d);
      g[r] = x[hi] - x[lo];
    }
    stage<H, 1>(g);
    if constexpr (H > 2) stage<H, 2>(g);
#pragma unroll
    for (int r = 0; r < H; ++r) {
      const int lo = insert0(r, d), hi = lo | (1 << d);
      g[r] *= (c[lo] + c[hi]);
    }
    stage<H, 1>(g);
    if constexpr (H > 2) stage<H, 2>(g);
#pragma unroll
    for (int r = 0; r < H; ++r) {
      const int lo = insert0(r, d), hi = lo | (1 << d);
      y[hi] += g[r];
      y[lo] -= g[r];
    }
  }
}

// Mass: y_a = sum_q detJ r_q N_a (N . x), r_q = rho(clamp(phi_q)) or 1.
template <int DIM, typename T, bool RHO>
__device__ __forceinline__ void elem_mass_coef(const T* ph, T A, T Bc, T* r) {
  constexpr int NC = 1 << DIM;
  if constexpr (RHO) {
#pragma unroll
    for (int i = 0; i < NC; ++i) r[i] = ph[i];
    all_stages<DIM>(r);
#pragma unroll
    for (int i = 0; i < NC; ++i) r[i] = __builtin_fma(A, clamp_t(r[i], T(NC)), Bc);
  } else {
#pragma unroll
    for (int i = 0; i < NC; ++i) r[i] = Bc;
  }
}
template <int DIM, typename T>
__device__ __forceinline__ void elem_mass_apply(const T* x, const T* r, T* y) {
  constexpr int NC = 1 << DIM;
#pragma unroll
  for (int i = 0; i < NC; ++i) y[i] = x[i];
  all_stages<DIM>(y);
#pragma unroll
  for (int i = 0; i < NC; ++i) y[i] *= r[i];
  all_stages<DIM>(y);
}

// ------------------------------------------------------------ op traits
enum OpKind { K_PP = 0, K_MASS = 1, K_MASS_RHO = 2 };
template <int OP, int DIM>
struct Traits;
template <int DIM>
struct Traits<K_PP, DIM> {
  static constexpr int NF = 1, NCF = 1;
  static constexpr bool MASK = false;
};
template <int DIM>
struct Traits<K_MASS, DIM> {
  static constexpr int NF = 1, NCF = 0;
  static constexpr bool MASK = false;
};
template <int DIM>
struct Traits<K_MASS_RHO, DIM> {
  static constexpr int NF = DIM, NCF = 1;
  static constexpr bool MASK = true;
};

template <typename T>
struct BrickArgs {
  const int32_t* table;
  const int8_t* level;
  const int16_t* rank;
  int64_t count;
  int64_t slot_base;
  int nbnd;
  int64_t n;        // field stride of x and y
  int64_t n_slots;  // field stride of slots
  const T* x;
  const T* coef;    // phase field phi~ (stride n) or null
  T* y;
  T* slots;
  const int32_t* hang;
  const uint8_t* wall;
  double alpha, beta;  // rho(phi) = alpha phi + beta
  double* partials;    // fused x.y partial per block, or null
  const int* done;
  // structured (uniform, lexicographically numbered) meshes: node indices are
  // computed from the brick anchor instead of read from the table
  const int32_t* anchor;  // 3 per brick, integer node coordinates
  int64_t sy, sz;         // index strides of y and z
  int32_t side;           // nodes per edge - 1
};

template <typename T, bool MASK>
__device__ __forceinline__ T fetch(const T* v, const uint8_t* wall, int32_t i) {
  if constexpr (MASK) return wall[i] ? T(0) : v[i];
  return v[i];
}
template <typename T, bool MASK>
__device__ __forceinline__ T gather(const T* v, const uint8_t* wall, const int32_t* hang, int32_t e) {
  if (e >= 0) return fetch<T, MASK>(v, wall, e);
  const int32_t* p = hang + 4 * (int64_t)(-e - 1);
  const int32_t p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3];
  if (p2 < 0) return (fetch<T, MASK>(v, wall, p0) + fetch<T, MASK>(v, wall, p1)) * T(0.5);
  return ((fetch<T, MASK>(v, wall, p0) + fetch<T, MASK>(v, wall, p1)) +
          (fetch<T, MASK>(v, wall, p2) + fetch<T, MASK>(v, wall, p3))) *
         T(0.25);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wavefront = BPB bricks; one lane = one leaf column of a brick, marching
// along the last axis.  WHOLE: every node of the brick is gathered into LDS
// up front (all loads in flight together); otherwise a three-layer LDS ring
// is refilled from registers two layers ahead.  STRUCT: uniform mesh with
// lexicographic node numbers, indices computed from the brick anchor.
template <int DIM, int B, typename T, int OP, bool WHOLE, bool STRUCT>
__global__ __launch_bounds__(64) void k_brick(BrickArgs<T> a) {
  using TR = Traits<OP, DIM>;
  constexpr int NF = TR::NF, NCF = TR::NCF, NV = NF + NCF;
  constexpr int LPB = DIM == 3 ? B * B : B;  // lanes (leaf columns) per brick
  constexpr int BPB = 64 / LPB;              // bricks per wavefront
  constexpr int NL = DIM == 3 ? (B + 1) * (B + 1) : (B + 1);  // nodes per layer
  constexpr int KL = (NL + LPB - 1) / LPB;   // layer nodes handled per lane
  constexpr int NC = 1 << DIM, NH = NC / 2;
  constexpr int RING = WHOLE ? B + 1 : 3;
  __shared__ T lay[RING][BPB][NV][NL];
  // per-corner-type leaf contributions, indexed by the node they land on
  // (zero where no leaf of the brick lands): a node sums NH entries
  __shared__ T accn[BPB][NF][NH][NL];
  if (a.done && *a.done) return;
  const int lane = threadIdx.x, bl = lane / LPB, ll = lane % LPB;
  const int64_t brick = (int64_t)blockIdx.x * BPB + bl;
  const bool active = brick < a.count;
  const int ix = ll % B, iy = DIM == 3 ? ll / B : 0;
  const int32_t* tab = a.table + (active ? brick : 0) * (int64_t)(NL * (B + 1));
  const int lev = active ? a.level[brick] : 0;
  int64_t base = 0;
  int32_t ax = 0, ay = 0, az = 0;
  if constexpr (STRUCT) {
    if (active) {
      ax = a.anchor[3 * brick];
      ay = a.anchor[3 * brick + 1];
      az = a.anchor[3 * brick + 2];
    }
    base = DIM == 3 ? ax + ay * a.sy + az * a.sz : ax + ay * a.sy;
  }
  // index of layer-z node p (STRUCT) or its table entry
  auto entry = [&](int z, int p) -> int64_t {
    if constexpr (STRUCT) {
      const int jx = p % (B + 1), jy = DIM == 3 ? p / (B + 1) : 0;
      return DIM == 3 ? base + jx + jy * a.sy + z * a.sz : base + jx + z * a.sy;
    } else {
      return tab[z * NL + p];
    }
  };
  auto on_wall = [&](int z, int p) -> bool {
    const int jx = p % (B + 1), jy = DIM == 3 ? p / (B + 1) : 0;
    const int cx = ax + jx, cy = DIM == 3 ? ay + jy : ay + z, cz = az + z;
    return cx == 0 || cx == a.side || cy == 0 || cy == a.side || (DIM == 3 && (cz == 0 || cz == a.side));
  };
  auto value = [&](int f, int64_t e, int z, int p) -> T {
    if constexpr (STRUCT) {
      if (f < NF) {
        if constexpr (TR::MASK) {
          if (on_wall(z, p)) return T(0);
        }
        return a.x[f * a.n + e];
      }
      return a.coef[(f - NF) * a.n + e];
    } else {
      if (f < NF) return gather<T, TR::MASK>(a.x + f * a.n, a.wall, a.hang, (int32_t)e);
      return gather<T, false>(a.coef + (f - NF) * a.n, nullptr, a.hang, (int32_t)e);
    }
  };
  // per-level folded constants (powers of two are exact); FP32 fields carry
  // 1 + phi, so rho = (beta - alpha) + alpha (1 + phi)
  const double beta0 = sizeof(T) == 8 ? a.beta : a.beta - a.alpha;
  T A = 0, Bc = 0;
  if constexpr (OP == K_PP) {
    // c~ = detJ (2/h)^2 / 4^d / rho = 1 / (rho / K); K = 2^{-(lev+1)(d-2) - 2d}
    const int e = (lev + 1) * (DIM - 2) + 2 * DIM;
    A = T(ldexp(a.alpha, e - DIM));
    Bc = T(ldexp(beta0, e));
  } else if constexpr (OP == K_MASS) {
    Bc = T(ldexp(1.0, -(lev + 1) * DIM - 2 * DIM));
  } else {
    const int e = -(lev + 1) * DIM - 2 * DIM;
    A = T(ldexp(a.alpha, e - DIM));
    Bc = T(ldexp(beta0, e));
  }

  // -------- layered pipeline state (entries three layers ahead, values two)
  int64_t ent[KL];
  T val[KL][NV];
  auto load_entries = [&](int z) {
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int p = ll + k * LPB;
      ent[k] = (active && z <= B && p < NL) ? entry(z, p) : 0;
    }
  };
  auto gather_vals = [&](int z) {
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int p = ll + k * LPB;
      if (active && z <= B && p < NL) {
#pragma unroll
        for (int f = 0; f < NV; ++f) val[k][f] = value(f, ent[k], z, p);
      }
    }
  };
  auto store_vals = [&](int z) {
    if (!active || z > B) return;
    const int buf = z % RING;
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int p = ll + k * LPB;
      if (p < NL)
#pragma unroll
        for (int f = 0; f < NV; ++f) lay[buf][bl][f][p] = val[k][f];
    }
  };

  double dot = 0.0;
  int64_t eo[KL];  // node indices of the layer being emitted (table meshes)
  auto load_emit_entries = [&](int z) {
    if constexpr (!STRUCT) {
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int p = ll + k * LPB;
        eo[k] = (active && p < NL) ? tab[z * NL + p] : 0;
      }
    }
  };
  auto emit_layer = [&](int z) {
    if (!active) return;
    const int buf = z % RING;
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int p = ll + k * LPB;
      if (p >= NL) continue;
      const int jx = p % (B + 1), jy = DIM == 3 ? p / (B + 1) : 0;
      T v[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        T t = accn[bl][f][0][p];
#pragma unroll
        for (int cl = 1; cl < NH; ++cl) t += accn[bl][f][cl][p];
        v[f] = t;
      }
      const bool interior = jx > 0 && jx < B && (DIM == 2 || (jy > 0 && jy < B)) && z > 0 && z < B;
      if (interior) {
        int64_t e;
        if constexpr (STRUCT) e = entry(z, p);
        else e = eo[k];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          a.y[f * a.n + e] = v[f];
          if (a.partials) dot += (double)lay[buf][bl][f][p] * (double)v[f];
        }
      } else {
        const int64_t sl = a.slot_base + brick * a.nbnd + brick_rank(DIM, B, jx, jy, z);
#pragma unroll
        for (int f = 0; f < NF; ++f) a.slots[f * a.n_slots + sl] = v[f];
      }
    }
  };

  T carry[NF][NH];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int c = 0; c < NH; ++c) carry[f][c] = T(0);

  if (active) {
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int p = ll + k * LPB;
      if (p < NL)
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int cl = 0; cl < NH; ++cl) accn[bl][f][cl][p] = T(0);
    }
  }
  if constexpr (WHOLE) {
    // every node of the brick: all loads issued before the first wait
    constexpr int NPB = NL * (B + 1);
    constexpr int KW = (NPB + LPB - 1) / LPB;
    if (active) {
      T w[KW][NV];
#pragma unroll
      for (int k = 0; k < KW; ++k) {
        const int q = ll + k * LPB;
        if (q < NPB) {
          const int z = q / NL, p = q % NL;
          const int64_t e = entry(z, p);
#pragma unroll
          for (int f = 0; f < NV; ++f) w[k][f] = value(f, e, z, p);
        }
      }
#pragma unroll
      for (int k = 0; k < KW; ++k) {
        const int q = ll + k * LPB;
        if (q < NPB)
#pragma unroll
          for (int f = 0; f < NV; ++f) lay[q / NL][bl][f][q % NL] = w[k][f];
      }
    }
  } else {
    // prologue: layers 0 and 1 into LDS, layer 2 in flight, entries of layer 3
    load_entries(0);
    gather_vals(0);
    store_vals(0);
    load_entries(1);
    gather_vals(1);
    store_vals(1);
    load_entries(2);
    gather_vals(2);
    load_entries(3);
  }
  __syncthreads();
  // corner values of the upper node layer of one leaf layer are the lower
  // corners of the next: keep them in registers and read only the new layer
  T xc[NF][NC], cc[NCF > 0 ? NCF : 1][NC];
  auto read_half = [&](int z, int half) {
#pragma unroll
    for (int c = 0; c < NH; ++c) {
      const int bx = c & 1, by = DIM == 3 ? (c >> 1) & 1 : 0;
      const int p = (ix + bx) + (DIM == 3 ? (iy + by) * (B + 1) : 0);
      const int buf = z % RING;
#pragma unroll
      for (int f = 0; f < NF; ++f) xc[f][c + half * NH] = lay[buf][bl][f][p];
#pragma unroll
      for (int f = 0; f < NCF; ++f) cc[f][c + half * NH] = lay[buf][bl][NF + f][p];
    }
  };
  if (active) read_half(0, 1);
  for (int ez = 0; ez < B; ++ez) {
    load_emit_entries(ez);
    if (active) {
      T ye[NF][NC];
#pragma unroll
      for (int c = 0; c < NH; ++c) {
#pragma unroll
        for (int f = 0; f < NF; ++f) xc[f][c] = xc[f][c + NH];
#pragma unroll
        for (int f = 0; f < NCF; ++f) cc[f][c] = cc[f][c + NH];
      }
      read_half(ez + 1, 1);
      if constexpr (OP == K_PP) {
        elem_pp<DIM, T>(xc[0], cc[0], A, Bc, ye[0]);
      } else {
        T r[NC];
        elem_mass_coef<DIM, T, OP == K_MASS_RHO>(cc[0], A, Bc, r);
#pragma unroll
        for (int f = 0; f < NF; ++f) elem_mass_apply<DIM, T>(xc[f], r, ye[f]);
      }
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int c = 0; c < NH; ++c) {
          const int p = (ix + (c & 1)) + (DIM == 3 ? (iy + ((c >> 1) & 1)) * (B + 1) : 0);
          accn[bl][f][c][p] = ye[f][c] + carry[f][c];
          carry[f][c] = ye[f][c + NH];
        }
    }
    __syncthreads();
    emit_layer(ez);
    if constexpr (!WHOLE) {
      store_vals(ez + 2);
      gather_vals(ez + 3);
      load_entries(ez + 4);
    }
    __syncthreads();
  }
  load_emit_entries(B);
  if (active) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int c = 0; c < NH; ++c) {
        const int p = (ix + (c & 1)) + (DIM == 3 ? (iy + ((c >> 1) & 1)) * (B + 1) : 0);
        accn[bl][f][c][p] = carry[f][c];
      }
  }
  __syncthreads();
  emit_layer(B);
  if (a.partials) {
    dot = wave_sum(dot);
    if (lane == 0) a.partials[blockIdx.x] = dot;
  }
}

// Block-wide deterministic sum of one double (256 threads).
__device__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

template <typename T, int NF, bool MASK>
__global__ __launch_bounds__(256) void k_combine(const int32_t* __restrict__ node, const int32_t* __restrict__ ptr,
                                                 const uint32_t* __restrict__ ent, int64_t nrows,
                                                 const T* __restrict__ slots, int64_t n_slots, T* __restrict__ y,
                                                 const T* __restrict__ x, int64_t n, const uint8_t* __restrict__ wall,
                                                 double* partials, const int* done) {
  __shared__ double sh[4];
  if (done && *done) return;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dot = 0.0;
  if (row < nrows) {
    const int32_t i = node[row];
    const int32_t k0 = ptr[row], k1 = ptr[row + 1];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      T v = T(0);
      for (int32_t k = k0; k < k1; ++k) {
        const uint32_t e = ent[k];
        const uint32_t code = e >> 30;
        const T s = slots[f * n_slots + (e & 0x3fffffffu)];
        v += code == 0 ? s : (code == 1 ? s * T(0.5) : s * T(0.25));
      }
      if constexpr (MASK) {
        if (wall[i]) v = x[f * n + i];
      }
      y[f * n + i] = v;
      if (partials) dot += (double)x[f * n + i] * (double)v;
    }
  }
  if (!partials) return;
  const double bs = block_sum256(dot, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// One block sums the per-block partials of the fused x.y in a fixed order
// (1024 threads, four independent running sums each).
__global__ __launch_bounds__(1024) void k_sum_partials(const double* partials, int n, double* out, const int* done) {
  __shared__ double sh[16];
  if (done && *done) return;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  int k = threadIdx.x;
  for (; k + 3 * 1024 < n; k += 4 * 1024) {
    v0 += partials[k];
    v1 += partials[k + 1024];
    v2 += partials[k + 2048];
    v3 += partials[k + 3072];
  }
  for (; k < n; k += 1024) v0 += partials[k];
  double v = wave_sum((v0 + v1) + (v2 + v3));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += sh[i];
    *out = t;
  }
}

// Wall rows of masked operators that no brick writes (all go through the
// combine, which handles them); nothing else is needed here.

// Diagonal probing helpers.
template <typename T>
__global__ void k_indicator(T* x, const uint8_t* color, int c, int64_t n, int nf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T v = color[i] == c ? T(1) : T(0);
  for (int f = 0; f < nf; ++f) x[f * n + i] = v;
}
template <typename T>
__global__ void k_take_diag(T* d, const T* y, const uint8_t* color, int c, int64_t n, int nf, int invert) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (color[i] != c) return;
  for (int f = 0; f < nf; ++f) {
    T v = y[f * n + i];
    d[f * n + i] = invert ? (v != T(0) ? T(1) / v : T(1)) : v;
  }
}

template <int DIM, int B, typename T, int OP>
constexpr bool whole_fits() {
  using TR = Traits<OP, DIM>;
  constexpr int LPB = DIM == 3 ? B * B : B;
  constexpr int NL = DIM == 3 ? (B + 1) * (B + 1) : (B + 1);
  // deep bricks keep the three-layer ring (better occupancy, loads pipelined)
  return B <= 4 && (64 / LPB) * NL * (B + 1) * (TR::NF + TR::NCF) * (int)sizeof(T) <= 12 * 1024;
}

template <int DIM, typename T, int OP, bool STRUCT>
void launch_b(int B, int64_t grid, hipStream_t s, const BrickArgs<T>& a) {
  const dim3 g((unsigned)grid), blk(64);
  switch (B) {
    case 8: k_brick<DIM, 8, T, OP, whole_fits<DIM, 8, T, OP>(), STRUCT><<<g, blk, 0, s>>>(a); break;
    case 4: k_brick<DIM, 4, T, OP, whole_fits<DIM, 4, T, OP>(), STRUCT><<<g, blk, 0, s>>>(a); break;
    case 2: k_brick<DIM, 2, T, OP, whole_fits<DIM, 2, T, OP>(), STRUCT><<<g, blk, 0, s>>>(a); break;
    default: k_brick<DIM, 1, T, OP, whole_fits<DIM, 1, T, OP>(), STRUCT><<<g, blk, 0, s>>>(a); break;
  }
}

template <int DIM, typename T, int OP>
int launch_bricks(const DevMesh& dm, BrickArgs<T> a, hipStream_t s, int& part_off) {
  for (int k = 0; k < kBrickClasses; ++k) {
    const DevBrickClass& bc = dm.cls[k];
    if (bc.count == 0) continue;
    a.table = bc.table;
    a.level = bc.level;
    a.rank = bc.rank;
    a.count = bc.count;
    a.slot_base = bc.slot_base;
    a.nbnd = bc.nbnd;
    double* part = a.partials;
    const int lpb = DIM == 3 ? bc.B * bc.B : bc.B;
    const int bpb = 64 / lpb;
    const int64_t grid = (bc.count + bpb - 1) / bpb;
    if (part) a.partials = part + part_off;
    if (dm.structured) {
      a.anchor = bc.anchor;
      launch_b<DIM, T, OP, true>(bc.B, grid, s, a);
    } else {
      launch_b<DIM, T, OP, false>(bc.B, grid, s, a);
    }
    CHNS_HIP(hipGetLastError());
    if (part) {
      part_off += (int)grid;
      a.partials = part;
    }
  }
  return CHNS_OK;
}

int64_t combine_blocks(const DevMesh& dm) { return (dm.n_comb + 255) / 256; }

template <int DIM, typename T, int OP>
int apply_t(Ctx& c, const LevelView& L, const T* x, T* y, const T* phi, hipStream_t s, const ApplyOut& o) {
  using TR = Traits<OP, DIM>;
  const DevMesh& dm = *L.dm;
  BrickArgs<T> a{};
  a.n = dm.n;
  a.n_slots = dm.n_slots;
  a.x = x;
  a.coef = phi;
  a.y = y;
  a.slots = (T*)L.slots;
  a.hang = dm.hang_par;
  a.wall = dm.wall;
  a.alpha = (c.prm.rho_plus - c.prm.rho_minus) / (2.0 * c.prm.rho_plus);
  a.beta = (c.prm.rho_plus + c.prm.rho_minus) / (2.0 * c.prm.rho_plus);
  a.partials = o.fuse_dot ? c.partials : nullptr;
  a.done = o.done;
  a.sy = dm.side + 1;
  a.sz = (int64_t)(dm.side + 1) * (dm.side + 1);
  a.side = dm.side;
  int part_off = 0;
  static const char* tags[3][2] = {{"pp_brick_fp64", "pp_brick_fp32"},
                                   {"mass_brick_fp64", "mass_brick_fp32"},
                                   {"massrho_brick_fp64", "massrho_brick_fp32"}};
  const char* tag = tags[OP][sizeof(T) == 8 ? 0 : 1];
  hipEvent_t ev;
  c.prof_begin(tag, s, &ev);
  int rc = launch_bricks<DIM, T, OP>(dm, a, s, part_off);
  if (rc) return rc;
  c.prof_end(tag, s, ev);
  const int64_t cb = combine_blocks(dm);
  const int total = part_off + (int)cb;
  if (o.fuse_dot && total > kMaxPartials) {
    set_error("mesh needs more reduction partials than allocated");
    return CHNS_EINVAL;
  }
  if (cb > 0 || o.fuse_dot) {
    const unsigned g = (unsigned)(cb > 0 ? cb : 1);
    c.prof_begin("combine", s, &ev);
    k_combine<T, TR::NF, TR::MASK><<<dim3(g), dim3(256), 0, s>>>(
        dm.comb_node, dm.comb_ptr, dm.comb_ent, dm.n_comb, (const T*)L.slots, dm.n_slots, y, x, dm.n, dm.wall,
        o.fuse_dot ? c.partials + part_off : nullptr, o.done);
    CHNS_HIP(hipGetLastError());
    c.prof_end("combine", s, ev);
  }
  if (o.fuse_dot) {
    k_sum_partials<<<1, 1024, 0, s>>>(c.partials, total, &c.sc->pq, o.done);
    CHNS_HIP(hipGetLastError());
  }
  return CHNS_OK;
}

template <typename T>
int apply_dispatch(Ctx& c, const LevelView& L, int op, const T* x, T* y, const T* phi, hipStream_t s,
                   const ApplyOut& o) {
  const int dim = L.dm->dim;
  switch (op) {
    case CHNS_OP_PRESSURE:
      return dim == 3 ? apply_t<3, T, K_PP>(c, L, x, y, phi, s, o) : apply_t<2, T, K_PP>(c, L, x, y, phi, s, o);
    case CHNS_OP_MASS:
      return dim == 3 ? apply_t<3, T, K_MASS>(c, L, x, y, phi, s, o) : apply_t<2, T, K_MASS>(c, L, x, y, phi, s, o);
    case CHNS_OP_MASS_RHO:
      return dim == 3 ? apply_t<3, T, K_MASS_RHO>(c, L, x, y, phi, s, o)
                      : apply_t<2, T, K_MASS_RHO>(c, L, x, y, phi, s, o);
  }
  set_error("operator not available");
  return CHNS_EINVAL;
}

}  // namespace

int op_fields(int op, int dim) {
  switch (op) {
    case CHNS_OP_PRESSURE:
    case CHNS_OP_MASS:
      return 1;
    case CHNS_OP_MASS_RHO:
    case CHNS_OP_MOMENTUM:
      return dim;
    case CHNS_OP_CH_JACOBIAN:
      return 2;
  }
  return 0;
}

LevelView fine_view(Ctx& c) { return LevelView{&c.dm, c.phi64, c.phi32, c.slots}; }

int launch_apply_lv(Ctx& c, const LevelView& L, int op, int prec, const void* x, void* y, hipStream_t s,
                    const ApplyOut& o) {
  if (op != CHNS_OP_MASS && !c.phi_set) {
    set_error("set_phase_field must be called before this operator");
    return CHNS_ESTATE;
  }
  if (prec == CHNS_FP64) return apply_dispatch<double>(c, L, op, (const double*)x, (double*)y, L.phi64, s, o);
  if (prec == CHNS_FP32) return apply_dispatch<float>(c, L, op, (const float*)x, (float*)y, L.phi32, s, o);
  set_error("prec must be CHNS_FP64 or CHNS_FP32");
  return CHNS_EINVAL;
}

int launch_apply(Ctx& c, int op, int prec, const void* x, void* y, hipStream_t s, const ApplyOut& o) {
  return launch_apply_lv(c, fine_view(c), op, prec, x, y, s, o);
}

// Exact diagonal of P^T K P by probing: colour classes never share a leaf
// (directly or through constraint parents), so y = A 1_c has y_i = A_ii on
// colour c.
int launch_diagonal_lv(Ctx& c, const LevelView& L, int op, int prec, void* d, bool invert, void* xi, void* yi,
                       hipStream_t s) {
  const int64_t n = L.dm->n;
  const int nf = op_fields(op, L.dm->dim);
  const unsigned g = (unsigned)((n + 255) / 256);
  ApplyOut o{};
  for (int col = 0; col < L.dm->n_colors; ++col) {
    if (prec == CHNS_FP64)
      k_indicator<double><<<g, 256, 0, s>>>((double*)xi, L.dm->color, col, n, nf);
    else
      k_indicator<float><<<g, 256, 0, s>>>((float*)xi, L.dm->color, col, n, nf);
    CHNS_HIP(hipGetLastError());
    int rc = launch_apply_lv(c, L, op, prec, xi, yi, s, o);
    if (rc) return rc;
    if (prec == CHNS_FP64)
      k_take_diag<double><<<g, 256, 0, s>>>((double*)d, (const double*)yi, L.dm->color, col, n, nf, invert);
    else
      k_take_diag<float><<<g, 256, 0, s>>>((float*)d, (const float*)yi, L.dm->color, col, n, nf, invert);
    CHNS_HIP(hipGetLastError());
  }
  return CHNS_OK;
}

int launch_diagonal(Ctx& c, int op, int prec, void* d, bool invert, hipStream_t s) {
  const int64_t n = c.dm.n;
  size_t es = prec == CHNS_FP64 ? 8 : 4;
  for (int k = 6; k < 8; ++k) {
    if (prec == CHNS_FP64 && !c.w64[k]) c.w64[k] = (double*)c.dalloc(es * n * 3);
    if (prec == CHNS_FP32 && !c.w32[k]) c.w32[k] = (float*)c.dalloc(es * n * 3);
    if ((prec == CHNS_FP64 && !c.w64[k]) || (prec == CHNS_FP32 && !c.w32[k])) return CHNS_ENOMEM;
  }
  void* xi = prec == CHNS_FP64 ? (void*)c.w64[6] : (void*)c.w32[6];
  void* yi = prec == CHNS_FP64 ? (void*)c.w64[7] : (void*)c.w32[7];
  return launch_diagonal_lv(c, fine_view(c), op, prec, d, invert, xi, yi, s);
}

}  // namespace chns
