// Geometric multigrid V-cycle for the pressure Poisson operator on octree
// levels.  The paper names geometric multigrid only as future work (its
// conclusions); it solves with algebraic multigrid instead.  Here every level
// is the octree truncated one level coarser (2:1 balance is kept), its
// operator is the same variable-coefficient apply rediscretised with the
// phase field injected from the finer level, the grid transfers are the
// exact Q1 embedding (hanging constraints of both levels included) and its
// transpose, smoothing is damped Jacobi with the exact diagonal, and the
// coarsest level (level 1: 27 nodes in 3D, 9 in 2D) is solved with a dense inverse of the
// operator regularised by (1/n) 1 1^T, which returns the mean-free solution
// for a right-hand side in the range.  The cycle is symmetric, so it is a
// fixed SPD preconditioner for CG.
//
// Uniform coarse levels (all of them below a uniform fine mesh, the levels
// at or below the minimum level of an adaptive one) hold their operator
// assembled as a 3^d-point stencil, computed once per phase field from the
// same element integrals (2-point Gauss, 1/rho of the clamped phase field at
// the Gauss points).  On them a smoothing sweep is one kernel (stencil
// product and Jacobi update together; the two pre-smoothing sweeps from a
// zero guess are one kernel), where the matrix-free path needs a brick
// launch, a combine launch and an update launch: on levels of a few
// thousand nodes every launch costs the same few microseconds, whatever its
// size.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>

#include "chns_internal.h"

namespace chns {
namespace {

constexpr int kT = 256;

inline unsigned blocks(int64_t n) {
  int64_t g = (n + kT - 1) / kT;
  if (g > 4096) g = 4096;
  return (unsigned)(g < 1 ? 1 : g);
}

// y = A x (accumulate: y += A x) for a CSR matrix with values of type V
template <typename T, typename V>
__global__ void k_spmv(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                       const V* __restrict__ val, const T* __restrict__ x, T* __restrict__ y, int64_t rows,
                       int accumulate) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < rows; i += (int64_t)gridDim.x * kT) {
    T acc = T(0);
    for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) acc += (T)val[k] * x[col[k]];
    y[i] = accumulate ? y[i] + acc : acc;
  }
}

// y = yin + A x (yin null: y = A x; yin may be y) with L lanes per row
// (lane-strided partial sums, then a fixed butterfly): coalesced reads of
// the column and value arrays
template <typename T, typename V, int L>
__global__ __launch_bounds__(kT) void k_spmv_g(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                               const V* __restrict__ val, const T* __restrict__ x, T* y,
                                               int64_t rows, const T* yin) {
  const int lane = threadIdx.x & (L - 1);
  const int64_t stride = (int64_t)gridDim.x * (kT / L);
  for (int64_t i = ((int64_t)blockIdx.x * kT + threadIdx.x) / L; i < rows; i += stride) {
    const int32_t b = ptr[i], e = ptr[i + 1];
    T acc = T(0);
    for (int32_t k = b + lane; k < e; k += L) acc += (T)val[k] * x[col[k]];
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
    if (lane == 0) y[i] = yin ? yin[i] + acc : acc;
  }
}

// z = w dinv r
template <typename T>
__global__ void k_jacobi0(T* z, const T* r, const T* dinv, T w, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    z[i] = w * dinv[i] * r[i];
}
template <typename T>
__global__ void k_copy_t(const T* a, T* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) b[i] = a[i];
}
// t = r - t
template <typename T>
__global__ void k_resid(const T* r, T* t, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) t[i] = r[i] - t[i];
}
// z = M r with a dense n x n row-major M
template <typename T>
__device__ __forceinline__ T dense_row(const T* M, const T* r, int i, int n) {
  T acc = T(0);
  for (int j = 0; j < n; ++j) acc += M[(int64_t)i * n + j] * r[j];
  return acc;
}
template <typename T>
__global__ void k_dense(const T* M, const T* r, T* z, int n) {
  for (int i = blockIdx.x * kT + threadIdx.x; i < n; i += gridDim.x * kT) z[i] = dense_row<T>(M, r, i, n);
}
// Structured transfers between uniform lexicographically numbered levels
// (fine side nf = 2 nc nodes per edge minus one): the Q1 embedding has weight
// 1 at coincident nodes and 1/2 per direction at midpoints.
//   restriction: coarse(I) = sum_{a in -1..1}^d w(a) (r - t)(2I + a)
//   prolongation: z(i) += coarse field at i
//   injection: coarse(I) = fine(2I)
// Neighbours outside the level get weight 0 at a clamped (valid) index, so
// that every load is unconditional and a thread issues all of them at once
// (on the small levels nothing else hides their latency); the added zeros
// leave the sums unchanged.
template <typename T, int DIM>
__device__ __forceinline__ T restrict_at(const T* __restrict__ r, const T* __restrict__ t, int64_t c, int nc) {
  const int nf = 2 * nc;
  const int64_t s1 = nc + 1, f1 = nf + 1;
  {
    const int I = (int)(c % s1), J = (int)((c / s1) % s1), K = DIM == 3 ? (int)(c / (s1 * s1)) : 0;
    T acc = T(0);
#pragma unroll
    for (int cz = (DIM == 3 ? -1 : 0); cz <= (DIM == 3 ? 1 : 0); ++cz) {
      const int k = 2 * K + cz;
      const T wz = (k < 0 || k > nf) ? T(0) : (cz ? T(0.5) : T(1));
      const int kk = min(max(k, 0), nf);
#pragma unroll
      for (int cy = -1; cy <= 1; ++cy) {
        const int j = 2 * J + cy;
        const T wy = (j < 0 || j > nf) ? T(0) : (cy ? wz * T(0.5) : wz);
        const int64_t row = ((int64_t)kk * f1 + min(max(j, 0), nf)) * f1;
#pragma unroll
        for (int cx = -1; cx <= 1; ++cx) {
          const int i = 2 * I + cx;
          const T w = (i < 0 || i > nf) ? T(0) : (cx ? wy * T(0.5) : wy);
          const int64_t ii = row + min(max(i, 0), nf);
          acc += w * (t ? r[ii] - t[ii] : r[ii]);
        }
      }
    }
    return acc;
  }
}
template <typename T, int DIM>
__global__ void k_restrict_s(const T* __restrict__ r, const T* __restrict__ t, T* __restrict__ out, int nc) {
  const int64_t s1 = nc + 1;
  const int64_t ncount = DIM == 3 ? s1 * s1 * s1 : s1 * s1;
  for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < ncount; c += (int64_t)gridDim.x * kT)
    out[c] = restrict_at<T, DIM>(r, t, c, nc);
}
// coarse-field value at fine node f (bilinear / trilinear interpolation)
template <typename T>
__device__ __forceinline__ T prolong_at(const T* __restrict__ zc, int64_t f, int nc, int dim) {
  const int64_t s1 = nc + 1, f1 = 2 * nc + 1;
  const int i = (int)(f % f1), j = (int)((f / f1) % f1), k = dim == 3 ? (int)(f / (f1 * f1)) : 0;
  const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
  auto at = [&](int a, int b, int c) { return zc[((int64_t)c * s1 + b) * s1 + a]; };
  if (dim == 3)
    return T(0.125) * ((at(i0, j0, k0) + at(i1, j0, k0)) + (at(i0, j1, k0) + at(i1, j1, k0)) +
                       (at(i0, j0, k1) + at(i1, j0, k1)) + (at(i0, j1, k1) + at(i1, j1, k1)));
  return T(0.25) * ((at(i0, j0, 0) + at(i1, j0, 0)) + (at(i0, j1, 0) + at(i1, j1, 0)));
}
template <typename T>
__global__ void k_prolong_s(const T* __restrict__ zc, const T* zin, T* zout, int nc, int dim) {
  const int64_t f1 = 2 * nc + 1;
  const int64_t fcount = dim == 3 ? f1 * f1 * f1 : f1 * f1;
  for (int64_t f = (int64_t)blockIdx.x * kT + threadIdx.x; f < fcount; f += (int64_t)gridDim.x * kT)
    zout[f] = zin[f] + prolong_at<T>(zc, f, nc, dim);  // zin may be zout
}
__global__ void k_inject_s(const double* __restrict__ fine, double* __restrict__ out, int nc, int dim) {
  const int64_t s1 = nc + 1, f1 = 2 * nc + 1;
  const int64_t ncount = dim == 3 ? s1 * s1 * s1 : s1 * s1;
  for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < ncount; c += (int64_t)gridDim.x * kT) {
    const int64_t I = c % s1, J = (c / s1) % s1, K = dim == 3 ? c / (s1 * s1) : 0;
    out[c] = fine[((2 * K) * f1 + 2 * J) * f1 + 2 * I];
  }
}

__global__ void k_unit(double* x, int j, int n) {
  for (int i = blockIdx.x * kT + threadIdx.x; i < n; i += gridDim.x * kT) x[i] = (i == j) ? 1.0 : 0.0;
}
__global__ void k_copy_col(const double* y, double* M, int j, int n) {
  for (int i = blockIdx.x * kT + threadIdx.x; i < n; i += gridDim.x * kT) M[(int64_t)j * n + i] = y[i];
}
__global__ void k_to32(const double* a, float* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) b[i] = (float)a[i];
}
__global__ void k_phase32(const double* a, float* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    b[i] = (float)(1.0 + a[i]);
}

// ---- assembled operators on uniform (structured) levels
// Elements of a uniform level with s cells per edge are numbered by anchor,
// x fastest; nodes i + (s+1) (j + (s+1) k).  Corner, Gauss point and child
// indices use bit d for axis d.  Element matrices (NC x NC, row-major):
//   K_ab = (h/2)^(d-2) sum_q c_q G_q(a, b),  G_q(a, b) = gradN_a . gradN_b at
//   the reference Gauss point q (+-1/sqrt 3 per axis), c_q = 1 / (alpha
//   clamp(phi_q, -1, 1) + beta), phi_q interpolated from the corners;
// a Galerkin coarse element (R A P with P the Q1 embedding, R = P^T) is
//   K_C = sum_children P_c^T K_c P_c, P_c(b, A) the weight of coarse corner A
//   at corner b of child c,
// which for children taken straight from the fine phase field is
//   K_C = (h_f/2)^(d-2) sum_{c,q} c_{c,q} H_{c,q},  H_{c,q} = P_c^T G_q P_c.
// Tables G (q, a, b), P (c, b, A) and H (c, q, A, B) are built on the host.

// Gauss-point coefficients of a level operator at the clamped phase value v:
// stiffness 1 / (a v + b) (pressure Poisson, 1/rho) or a v + b (one velocity
// component of the momentum operator, eta/(2 Re)); mass ma v + mb (a
// constant shift, or rho/dt)
struct QCoef {
  double a, b, ma, mb;
  int lin;
  __device__ __forceinline__ double k(double v) const { return lin ? a * v + b : rcp(a * v + b); }
  // hardware reciprocal estimate refined by two Newton steps
  __device__ __forceinline__ static double rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
  }
  __device__ __forceinline__ double m(double v) const { return ma * v + mb; }
};

__device__ __forceinline__ double phase_at(const double* ph, int q, int dim) {
  // phase field at reference Gauss point q from the corner values
  const double g = 0.57735026918962576451;
  const int nc = 1 << dim;
  double v = 0.0;
  for (int b = 0; b < nc; ++b) {
    double w = 1.0;
    for (int d = 0; d < dim; ++d) {
      const double sb = ((b >> d) & 1) ? 1.0 : -1.0, xq = ((q >> d) & 1) ? g : -g;
      w *= 0.5 * (1.0 + sb * xq);
    }
    v += w * ph[b];
  }
  return fmin(fmax(v, -1.0), 1.0);
}

// element matrices of a uniform level from its own phase field
// (one wave per element, lane (a, b) one entry)
template <int DIM>
__global__ __launch_bounds__(64) void k_el_rediscr(const double* __restrict__ phi, int s, const double* __restrict__ Gt,
                                                   QCoef cf, double scale, double* E, const double* __restrict__ Mq,
                                                   double mscale) {
  constexpr int NC = 1 << DIM, NE = NC * NC;
  __shared__ double cq[NC], cm[NC];
  const int64_t e = blockIdx.x;
  const int64_t s1 = s + 1;
  const int X = (int)(e % s), Y = (int)((e / s) % s), Z = DIM == 3 ? (int)(e / ((int64_t)s * s)) : 0;
  const int t = threadIdx.x;
  if (t < NC) {
    double ph[NC];
    for (int b = 0; b < NC; ++b)
      ph[b] = phi[((int64_t)(Z + ((b >> 2) & 1)) * s1 + (Y + ((b >> 1) & 1))) * s1 + (X + (b & 1))];
    const double v = phase_at(ph, t, DIM);
    cq[t] = cf.k(v);
    cm[t] = cf.m(v);
  }
  __syncthreads();
  if (t < NE) {
    double acc = 0.0, macc = 0.0;
    for (int q = 0; q < NC; ++q) {
      acc += cq[q] * Gt[q * NE + t];
      macc += cm[q] * Mq[q * NE + t];
    }
    E[e * NE + t] = scale * acc + mscale * macc;
  }
}

// Order the LDS traffic between the lanes of a one-wave workgroup: a wave's
// LDS operations complete in issue order, so fences at wavefront scope
// around a compiler-level wave barrier suffice; unlike __syncthreads this
// does not wait for the wave's global loads and stores still in flight.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Galerkin element matrices of a uniform level (sc cells per edge) straight
// from the phase field of the uniform level above (sf = 2 sc).  One wave
// handles kGalPerWave coarse elements; lane t keeps column t of H (the 64
// table entries it needs) in registers across them.  A constant mass
// (VARM false) is the coarse mass times mconst; a variable one (rho/dt) is
// the Galerkin product of the fine Gauss-point masses, sum cm_{c,q} Hm_{c,q}
// scaled by the fine det J (Hm staged in LDS).
constexpr int kGalPerWave = 64;
//
// The same pass also yields the fine level's diagonal: lane (c, u) forms
// child c's diagonal entry at its corner u from the child's Gauss-point
// coefficients (the G_q(u, u) and Mq_q(u, u) tables), the 3^d fine nodes of
// the coarse element sum their contributions in a fixed order into DP
// (3^d partials per coarse element), and k_diag_gather adds the partials of
// the coarse elements around each fine node.
template <int DIM, bool VARM>
__global__ __launch_bounds__(64) void k_gal_phi(const double* __restrict__ phi, int sf, const double* __restrict__ Ht,
                                                QCoef cf, double scale, double* E, int64_t ne,
                                                const double* __restrict__ Mt, double mconst,
                                                const double* __restrict__ Hm, double mscale,
                                                const double* __restrict__ Gt, const double* __restrict__ Mq,
                                                double fmscale, double* DP) {
  constexpr int NC = 1 << DIM, NE = NC * NC, NB = DIM == 3 ? 27 : 9;
  __shared__ double cq[NE], cm[NE], hm[VARM ? NE * NE : 1], dd[NE], pv[kGalPerWave * NB];
  const int sc = sf / 2;
  const int64_t f1 = sf + 1;
  const int t = threadIdx.x;
  double h[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) h[k] = t < NE ? Ht[k * NE + t] : 0.0;
  // the mass part of a shifted operator is reproduced exactly by the
  // Galerkin product (Q1 spaces are nested, 2-point Gauss is exact for it)
  const double m = t < NE ? mconst * Mt[t] : 0.0;
  if constexpr (VARM) {
    // eight loads in flight at a time
    for (int k0 = 0; k0 < NE * NE; k0 += 8 * 64) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = k0 + 64 * u + t < NE * NE ? Hm[k0 + 64 * u + t] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + 64 * u + t < NE * NE) hm[k0 + 64 * u + t] = v[u];
    }
  }
  // lane t: child c = t / NC, Gauss point q = t % NC of that child
  const int c = t / NC, q = t % NC;
  // diagonal tables of corner u = t % NC (lane t = (child, corner) in the
  // diagonal pass)
  double gd[NC], md[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    gd[k] = t < NE ? Gt[k * NE + q * NC + q] : 0.0;
    md[k] = t < NE ? Mq[k * NE + q * NC + q] : 0.0;
  }
  // one element with the phase values ph of its children's corners
  auto element = [&](int64_t e, const double* ph) {
    if (t < NE) {
      const double v = phase_at(ph, q, DIM);
      cq[t] = cf.k(v);
      cm[t] = cf.m(v);
    }
    wave_sync();
    if (t < NE) {
      // child c = t / NC, corner u = t % NC: that child's diagonal entry there
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        a += cq[c * NC + k] * gd[k];
        b += cm[c * NC + k] * md[k];
      }
      dd[t] = scale * a + fmscale * b;
    }
    wave_sync();
    if (t < NB) {
      // local fine node (i, j, k) in {0, 1, 2}^d: children and corners with
      // c_d + u_d = i_d (child c spans fine cells c_d .. c_d + 1), in a
      // fixed order
      const int li[3] = {t % 3, (t / 3) % 3, DIM == 3 ? t / 9 : 0};
      double s = 0.0;
      for (int cz = 0; cz < (DIM == 3 ? 2 : 1); ++cz)
        for (int cy = 0; cy < 2; ++cy)
          for (int cx = 0; cx < 2; ++cx) {
            const int ux = li[0] - cx, uy = li[1] - cy, uz = li[2] - cz;
            if (ux < 0 || ux > 1 || uy < 0 || uy > 1 || uz < 0 || uz > 1) continue;
            s += dd[(cx + 2 * cy + 4 * cz) * NC + (ux + 2 * uy + 4 * uz)];
          }
      DP[e * NB + t] = s;
    }
    if (t < NE) {
      // four independent partial sums: a 64-long dependent chain would
      // dominate the per-element latency
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < NE; ++k) a4[k & 3] += cq[k] * h[k];
      const double acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
      if constexpr (VARM) {
        double macc = 0.0;
        for (int k = 0; k < NE; ++k) macc += cm[k] * hm[k * NE + t];
        E[e * NE + t] = scale * acc + mscale * macc;
      } else {
        E[e * NE + t] = scale * acc + m;
      }
    }
    wave_sync();
  };
  // the phase values at the 3^d fine nodes of each of the wave's elements,
  // staged in LDS with all loads in flight at once; the element loop then
  // issues no global loads (a register prefetch of the next element made the
  // wave wait for its loads at once)
  const int64_t e0 = (int64_t)blockIdx.x * kGalPerWave;
  const int64_t e1 = e0 + kGalPerWave < ne ? e0 + kGalPerWave : ne;
  const int nel = (int)(e1 - e0);
  {
    // sc = 2^ls (a uniform level): element coordinates by shifts
    const int ls = __builtin_ctz((unsigned)sc);
    double v[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int idx = t + 64 * r;
      v[r] = 0.0;
      if (idx < nel * NB) {
        const int64_t e = e0 + idx / NB;
        const int nd = idx % NB;
        const int X = (int)(e & (sc - 1)), Y = (int)((e >> ls) & (sc - 1)), Z = DIM == 3 ? (int)(e >> (2 * ls)) : 0;
        const int lx = nd % 3, ly = (nd / 3) % 3, lz = DIM == 3 ? nd / 9 : 0;
        v[r] = phi[((int64_t)(2 * Z + lz) * f1 + (2 * Y + ly)) * f1 + (2 * X + lx)];
      }
    }
#pragma unroll
    for (int r = 0; r < NB; ++r)
      if (t + 64 * r < nel * NB) pv[t + 64 * r] = v[r];
  }
  wave_sync();
  for (int64_t e = e0; e < e1; ++e) {
    // child c's corner b is fine node (c_d + b_d)_d of the element's 3^d
    const double* pe = pv + (e - e0) * NB;
    double ph[NC];
#pragma unroll
    for (int b = 0; b < NC; ++b)
      ph[b] = pe[((c & 1) + (b & 1)) + 3 * (((c >> 1) & 1) + ((b >> 1) & 1)) +
                 (DIM == 3 ? 9 * (((c >> 2) & 1) + ((b >> 2) & 1)) : 0)];
    element(e, ph);
  }
}

// inverse diagonal of the fine level from the per-coarse-element partials
// of k_gal_phi: the partials of the (up to 2^d) coarse elements around each
// fine node, in a fixed order
template <int DIM>
__global__ void k_diag_gather(const double* __restrict__ DP, int sc, double* dinv64, float* dinv32) {
  constexpr int NB = DIM == 3 ? 27 : 9;
  const int sf = 2 * sc;
  const int64_t f1 = sf + 1;
  const int64_t n = DIM == 3 ? f1 * f1 * f1 : f1 * f1;
  for (int64_t node = (int64_t)blockIdx.x * kT + threadIdx.x; node < n; node += (int64_t)gridDim.x * kT) {
    const int P[3] = {(int)(node % f1), (int)((node / f1) % f1), DIM == 3 ? (int)(node / (f1 * f1)) : 0};
    // per axis: (coarse index, local index) options
    int ce[3][2], lo[3][2], no[3];
    for (int d = 0; d < 3; ++d) {
      no[d] = 0;
      if (d >= DIM) {
        ce[d][0] = 0;
        lo[d][0] = 0;
        no[d] = 1;
        continue;
      }
      if (P[d] % 2) {
        ce[d][0] = (P[d] - 1) / 2;
        lo[d][0] = 1;
        no[d] = 1;
      } else {
        if (P[d] / 2 - 1 >= 0) {
          ce[d][no[d]] = P[d] / 2 - 1;
          lo[d][no[d]++] = 2;
        }
        if (P[d] / 2 < sc) {
          ce[d][no[d]] = P[d] / 2;
          lo[d][no[d]++] = 0;
        }
      }
    }
    double acc = 0.0;
    for (int kz = 0; kz < no[2]; ++kz)
      for (int ky = 0; ky < no[1]; ++ky)
        for (int kx = 0; kx < no[0]; ++kx) {
          const int64_t e = ce[0][kx] + (int64_t)sc * (ce[1][ky] + (DIM == 3 ? (int64_t)sc * ce[2][kz] : 0));
          acc += DP[e * NB + lo[0][kx] + 3 * lo[1][ky] + 9 * lo[2][kz]];
        }
    dinv64[node] = 1.0 / acc;
    dinv32[node] = (float)(1.0 / acc);
  }
}

// Galerkin element matrices of a uniform level from the element matrices of
// the uniform level above: K_C = sum_c P_c^T K_c P_c (fixed child order)
template <int DIM>
__global__ __launch_bounds__(64) void k_gal_elem(const double* __restrict__ Ef, int sf, const double* __restrict__ Pt,
                                                 double* E) {
  constexpr int NC = 1 << DIM, NE = NC * NC;
  // all children at once: K_c and T_c = K_c P_c for every child in LDS, two
  // barriers per coarse element (the same sums in the same order as child
  // by child)
  __shared__ double K[NC * NE], T[NC * NE], Ps[NC * NE];
  const int64_t e = blockIdx.x;
  const int sc = sf / 2;
  const int X = (int)(e % sc), Y = (int)((e / sc) % sc), Z = DIM == 3 ? (int)(e / ((int64_t)sc * sc)) : 0;
  const int t = threadIdx.x;
  const int r = t / NC, col = t % NC;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t ce = (2 * X + (c & 1)) + (int64_t)sf * ((2 * Y + ((c >> 1) & 1)) +
                                                          (DIM == 3 ? (int64_t)sf * (2 * Z + ((c >> 2) & 1)) : 0));
    if (t < NE) K[c * NE + t] = Ef[ce * NE + t];
  }
  for (int k = t; k < NC * NE; k += 64) Ps[k] = Pt[k];
  __syncthreads();
  // T_c(b = r, B = col) = sum_b2 K_c(r, b2) P_c(b2, col)
  if (t < NE)
    for (int c = 0; c < NC; ++c) {
      double v = 0.0;
      for (int b2 = 0; b2 < NC; ++b2) v += K[c * NE + r * NC + b2] * Ps[(c * NC + b2) * NC + col];
      T[c * NE + t] = v;
    }
  __syncthreads();
  // K_C(A = r, B = col) = sum_c sum_b P_c(b, A) T_c(b, B)
  if (t < NE) {
    double acc = 0.0;
    for (int c = 0; c < NC; ++c)
      for (int b = 0; b < NC; ++b) acc += Ps[(c * NC + b) * NC + r] * T[c * NE + b * NC + col];
    E[e * NE + t] = acc;
  }
}

// 3^d-point stencil (and inverse diagonal) of a uniform level from its
// element matrices: node row = sum over the leaves around the node of the
// leaf matrix row of the corner the node occupies (fixed leaf order)
template <int DIM>
__global__ void k_el_stencil(const double* __restrict__ E, int s, double* S64, float* S32, double* dinv64,
                             float* dinv32) {
  constexpr int NC = 1 << DIM, NE = NC * NC, NS = DIM == 3 ? 27 : 9;
  const int64_t s1 = s + 1;
  const int64_t n = DIM == 3 ? s1 * s1 * s1 : s1 * s1;
  for (int64_t node = (int64_t)blockIdx.x * kT + threadIdx.x; node < n; node += (int64_t)gridDim.x * kT) {
    const int I = (int)(node % s1), J = (int)((node / s1) % s1), K = DIM == 3 ? (int)(node / (s1 * s1)) : 0;
    double acc[NS];
#pragma unroll
    for (int o = 0; o < NS; ++o) acc[o] = 0.0;
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      // the node is the upper corner of the leaf along axis d where bit d of u is set
      const int ux = u & 1, uy = (u >> 1) & 1, uz = DIM == 3 ? (u >> 2) & 1 : 0;
      const int ax = I - ux, ay = J - uy, az = K - uz;
      if (ax < 0 || ax >= s || ay < 0 || ay >= s || (DIM == 3 && (az < 0 || az >= s))) continue;
      const int64_t e = ax + (int64_t)s * (ay + (DIM == 3 ? (int64_t)s * az : 0));
      const double* row = E + e * NE + u * NC;
#pragma unroll
      for (int b = 0; b < NC; ++b) {
        const int ox = (b & 1) - ux, oy = ((b >> 1) & 1) - uy, oz = DIM == 3 ? ((b >> 2) & 1) - uz : 0;
        acc[(ox + 1) + 3 * (oy + 1) + (DIM == 3 ? 9 * (oz + 1) : 0)] += row[b];
      }
    }
#pragma unroll
    for (int o = 0; o < NS; ++o) {
      if (S64) S64[o * n + node] = acc[o];
      if (S32) S32[o * n + node] = (float)acc[o];
    }
    constexpr int C = NS / 2;
    if (dinv64) dinv64[node] = 1.0 / acc[C];
    if (dinv32) dinv32[node] = (float)(1.0 / acc[C]);
  }
}

// dense n x n matrix (row-major) of a uniform level's stencil
template <int DIM>
__global__ void k_stencil_dense(const double* __restrict__ S, int s, double* M) {
  constexpr int NS = DIM == 3 ? 27 : 9;
  const int64_t s1 = s + 1;
  const int64_t n = DIM == 3 ? s1 * s1 * s1 : s1 * s1;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const int I = (int)(i % s1), J = (int)((i / s1) % s1), K = DIM == 3 ? (int)(i / (s1 * s1)) : 0;
    for (int64_t j = 0; j < n; ++j) M[i * n + j] = 0.0;
    for (int o = 0; o < NS; ++o) {
      const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = DIM == 3 ? o / 9 - 1 : 0;
      if (I + ox < 0 || I + ox > s || J + oy < 0 || J + oy > s) continue;
      if (DIM == 3 && (K + oz < 0 || K + oz > s)) continue;
      M[i * n + (i + ox + oy * s1 + (DIM == 3 ? oz * s1 * s1 : 0))] = S[o * n + i];
    }
  }
}

// sum_o S_o(i) v(i + off_o) on a uniform level (zero stencil entries reach
// no node outside the level; their indices are skipped)
//
// Index of the neighbour at offset (ox, oy, oz), clamped into the level: the
// stencil value of an offset outside the level is 0, so every load can be
// unconditional (all issued at once) and the sum is the same.
template <int DIM>
__device__ __forceinline__ int64_t nbr(int64_t node, int ox, int oy, int oz, int64_t s1, int64_t n) {
  const int64_t j = node + ox + oy * s1 + (DIM == 3 ? oz * s1 * s1 : 0);
  return j < 0 ? 0 : (j >= n ? n - 1 : j);
}
template <typename T, int DIM, typename ST>
__device__ __forceinline__ T stencil_row(const ST* __restrict__ S, const T* __restrict__ v, int64_t node, int64_t n,
                                         int I, int J, int K, int s) {
  const int64_t s1 = s + 1;
  T acc = T(0);
#pragma unroll
  for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz) {
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy) {
#pragma unroll
      for (int ox = -1; ox <= 1; ++ox) {
        const int o = (ox + 1) + 3 * (oy + 1) + (DIM == 3 ? 9 * (oz + 1) : 0);
        acc += (T)S[o * n + node] * v[nbr<DIM>(node, ox, oy, oz, s1, n)];
      }
    }
  }
  return acc;
}
template <int DIM>
__device__ __forceinline__ void node_ijk(int64_t node, int s, int& I, int& J, int& K) {
  const int64_t s1 = s + 1;
  I = (int)(node % s1);
  J = (int)((node / s1) % s1);
  K = DIM == 3 ? (int)(node / (s1 * s1)) : 0;
}
// Per-node bodies of the stencil smoothers, shared by the per-level kernels
// below and the fused coarse tail (the same arithmetic in both).
// (A w D^-1 r)(i): the image of the first damped-Jacobi sweep from z = 0
template <typename T, int DIM, typename ST>
__device__ __forceinline__ T first_sweep_image(const ST* __restrict__ S, const T* __restrict__ dinv,
                                               const T* __restrict__ r, T w, int64_t i, int s, int64_t n) {
  const int64_t s1 = s + 1;
  T az = T(0);
#pragma unroll
  for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz) {
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy) {
#pragma unroll
      for (int ox = -1; ox <= 1; ++ox) {
        const int o = (ox + 1) + 3 * (oy + 1) + (DIM == 3 ? 9 * (oz + 1) : 0);
        const int64_t j = nbr<DIM>(i, ox, oy, oz, s1, n);
        az += (T)S[o * n + i] * (w * dinv[j] * r[j]);
      }
    }
  }
  return az;
}
// two sweeps from z = 0 at node i: z1 + w D^-1 (r - A z1) with z1 = w D^-1 r
template <typename T, int DIM, typename ST>
__device__ __forceinline__ T pre2_at(const ST* __restrict__ S, const T* __restrict__ dinv, const T* __restrict__ r,
                                     T w, int64_t i, int s, int64_t n) {
  const T az = first_sweep_image<T, DIM, ST>(S, dinv, r, w, i, s, n);
  const T z1 = w * dinv[i] * r[i];
  return z1 + w * dinv[i] * (r[i] - az);
}
// one sweep from zi at node i: zi + w D^-1 (r - A zi)
template <typename T, int DIM, typename ST>
__device__ __forceinline__ T sweep_at(const ST* __restrict__ S, const T* __restrict__ dinv, const T* __restrict__ r,
                                      const T* __restrict__ zi, T w, int64_t i, int s, int64_t n) {
  int I, J, K;
  node_ijk<DIM>(i, s, I, J, K);
  return zi[i] + w * dinv[i] * (r[i] - stencil_row<T, DIM, ST>(S, zi, i, n, I, J, K, s));
}
template <typename T, int DIM, typename ST>
__device__ __forceinline__ T row_at(const ST* __restrict__ S, const T* __restrict__ z, int64_t i, int s, int64_t n) {
  int I, J, K;
  node_ijk<DIM>(i, s, I, J, K);
  return stencil_row<T, DIM, ST>(S, z, i, n, I, J, K, s);
}
// two damped-Jacobi sweeps from z = 0: z1 = w D^-1 r, z2 = z1 + w D^-1 (r - A z1)
template <typename T, int DIM, typename ST>
__global__ void k_st_pre2(const ST* __restrict__ S, const T* __restrict__ dinv, const T* __restrict__ r,
                          T* __restrict__ z, T w, int s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    z[i] = pre2_at<T, DIM, ST>(S, dinv, r, w, i, s, n);
}
// one damped-Jacobi sweep from z = 0 and its image: z = w D^-1 r, t = A z
template <typename T, int DIM, typename ST>
__global__ void k_st_pre1(const ST* __restrict__ S, const T* __restrict__ dinv, const T* __restrict__ r,
                          T* __restrict__ z, T* __restrict__ t, T w, int s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    z[i] = w * dinv[i] * r[i];
    t[i] = first_sweep_image<T, DIM, ST>(S, dinv, r, w, i, s, n);
  }
}
// zo = zi + w D^-1 (r - A zi)
template <typename T, int DIM, typename ST>
__global__ void k_st_sweep(const ST* __restrict__ S, const T* __restrict__ dinv, const T* __restrict__ r,
                           const T* __restrict__ zi, T* __restrict__ zo, T w, int s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    zo[i] = sweep_at<T, DIM, ST>(S, dinv, r, zi, w, i, s, n);
}
// t = A z
template <typename T, int DIM, typename ST>
__global__ void k_st_apply(const ST* __restrict__ S, const T* __restrict__ z, T* __restrict__ t, int s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    t[i] = row_at<T, DIM, ST>(S, z, i, s, n);
}

// The coarse tail of the stencil V-cycle in one workgroup, held in LDS: the
// levels at the bottom of the hierarchy (9^3 nodes and coarser in 3D) and
// the dense coarsest level fit in one CU's 160 KiB of LDS together with
// their stencils.  One launch stages the stencils, diagonals, coarsest
// inverse and the first level's right-hand side into LDS, runs every phase
// of the cycle from there down and back up (one loop over a level's nodes
// per phase, a workgroup barrier between phases) and writes the first
// level's correction back.  The per-level kernels above take one launch per
// phase instead (ten for this part of the level-7 pressure cycle, each a few
// microseconds of launch and memory latency over a few hundred nodes).
// Same per-node arithmetic in the same order, so the same results.
constexpr int kTailT = 1024;
constexpr int kTailLevels = 8;
constexpr int kTailLds = 160 * 1024;  // bytes
template <typename T>
struct TailLevel {
  const float* S;  // global: stencil, diagonal, and for the first level the correction
  const T* dinv;
  T* z;
  int side, n;
  int oS, od, orr, oz, ot, oz2;  // byte offsets of the LDS copies
};
// one staged region: bytes (a multiple of 4) from global src to LDS offset
// dst; chunk0 = its first 16-byte chunk in the staging order
struct TailSeg {
  const char* src;
  int dst, bytes, chunk0;
};
constexpr int kTailSegs = 2 * kTailLevels + 2;
constexpr int kTailU = 8;  // 16-byte chunks per thread per staging trip
template <typename T>
struct TailArgs {
  TailSeg seg[kTailSegs];
  int nseg, nchunk;
  TailLevel<T> lv[kTailLevels];
  int nl;        // stencil levels
  const T* inv;  // coarsest level: dense inverse (global)
  int sideK, nK;
  int oinv, orK, ozK;
  int nu;
  T w;
};
template <typename T, int DIM>
__global__ __launch_bounds__(kTailT) void k_vcycle_tail(const TailArgs<T> a) {
  __shared__ double lds[kTailLds / sizeof(double)];
  char* base = reinterpret_cast<char*>(lds);
  const int tid = threadIdx.x;
  constexpr int NS = DIM == 3 ? 27 : 9;
  auto F = [&](int off) { return reinterpret_cast<float*>(base + off); };
  auto V = [&](int off) { return reinterpret_cast<T*>(base + off); };
  // staging: the whole 16-byte chunks of every region, kTailU per thread
  // with all loads in flight before the stores, then the last 4-byte words
  for (int c0 = tid; c0 < a.nchunk; c0 += kTailU * kTailT) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    v4i v[kTailU];
    int dst[kTailU];
#pragma unroll
    for (int u = 0; u < kTailU; ++u) {
      const int ch = c0 + u * kTailT;
      dst[u] = -1;
      if (ch < a.nchunk) {
        int g = 0;  // the last region starting at or before chunk ch
#pragma unroll
        for (int q = 1; q < kTailSegs; ++q) g += (q < a.nseg && a.seg[q].chunk0 <= ch) ? 1 : 0;
        const int k = ch - a.seg[g].chunk0;
        v[u] = reinterpret_cast<const v4i*>(a.seg[g].src)[k];
        dst[u] = a.seg[g].dst + 16 * k;
      }
    }
#pragma unroll
    for (int u = 0; u < kTailU; ++u)
      if (dst[u] >= 0) *reinterpret_cast<v4i*>(base + dst[u]) = v[u];
  }
  for (int g = 0; g < a.nseg; ++g) {
    const int whole = a.seg[g].bytes / 16 * 16;
    if (tid < (a.seg[g].bytes - whole) / 4)
      reinterpret_cast<int*>(base + a.seg[g].dst + whole)[tid] =
          reinterpret_cast<const int*>(a.seg[g].src + whole)[tid];
  }
  __syncthreads();
  for (int l = 0; l < a.nl; ++l) {
    const TailLevel<T>& L = a.lv[l];
    const float* S = F(L.oS);
    const T* dinv = V(L.od);
    const T* r = V(L.orr);
    T* z = V(L.oz);
    T* t = V(L.ot);
    T* z2 = V(L.oz2);
    const int64_t n = L.n;
    if (a.nu == 1) {
      for (int64_t i = tid; i < n; i += kTailT) {
        z[i] = a.w * dinv[i] * r[i];
        t[i] = first_sweep_image<T, DIM, float>(S, dinv, r, a.w, i, L.side, n);
      }
    } else {
      for (int64_t i = tid; i < n; i += kTailT) z[i] = pre2_at<T, DIM, float>(S, dinv, r, a.w, i, L.side, n);
      for (int it = 2; it < a.nu; ++it) {
        __syncthreads();
        for (int64_t i = tid; i < n; i += kTailT) z2[i] = sweep_at<T, DIM, float>(S, dinv, r, z, a.w, i, L.side, n);
        __syncthreads();
        for (int64_t i = tid; i < n; i += kTailT) z[i] = z2[i];
      }
      __syncthreads();
      for (int64_t i = tid; i < n; i += kTailT) t[i] = row_at<T, DIM, float>(S, z, i, L.side, n);
    }
    __syncthreads();
    const bool last = l + 1 == a.nl;
    T* rc = V(last ? a.orK : a.lv[l + 1].orr);
    const int sc = last ? a.sideK : a.lv[l + 1].side;
    const int64_t nc = last ? a.nK : a.lv[l + 1].n;
    for (int64_t c = tid; c < nc; c += kTailT) rc[c] = restrict_at<T, DIM>(r, t, c, sc);
    __syncthreads();
  }
  {
    const T* M = V(a.oinv);
    const T* rK = V(a.orK);
    T* zK = V(a.ozK);
    for (int i = tid; i < a.nK; i += kTailT) zK[i] = dense_row<T>(M, rK, i, a.nK);
  }
  __syncthreads();
  const bool odd = a.nu % 2 == 1;
  for (int l = a.nl - 1; l >= 0; --l) {
    const TailLevel<T>& L = a.lv[l];
    const float* S = F(L.oS);
    const T* dinv = V(L.od);
    const T* r = V(L.orr);
    T* z = V(L.oz);
    const int64_t n = L.n;
    const bool last = l + 1 == a.nl;
    const T* zc = V(last ? a.ozK : a.lv[l + 1].oz);
    const int sc = last ? a.sideK : a.lv[l + 1].side;
    // for odd nu the prolongation writes to z2, so the sweeps end in z
    T* cur = odd ? V(L.oz2) : z;
    T* oth = odd ? z : V(L.oz2);
    for (int64_t f = tid; f < n; f += kTailT) cur[f] = z[f] + prolong_at<T>(zc, f, sc, DIM);
    for (int it = 0; it < a.nu; ++it) {
      __syncthreads();
      for (int64_t i = tid; i < n; i += kTailT) oth[i] = sweep_at<T, DIM, float>(S, dinv, r, cur, a.w, i, L.side, n);
      T* x = cur;
      cur = oth;
      oth = x;
    }
    __syncthreads();
  }
  const T* z0 = V(a.lv[0].oz);
  for (int i = tid; i < a.lv[0].n; i += kTailT) a.lv[0].z[i] = z0[i];
}

template <typename T>
int upload(Ctx& c, T** dst, const std::vector<T>& src) {
  *dst = (T*)c.dalloc(sizeof(T) * (src.empty() ? 1 : src.size()));
  if (!*dst) return CHNS_ENOMEM;
  if (!src.empty()) CHNS_HIP(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
  return CHNS_OK;
}
template <typename T>
int upload_as_float(Ctx& c, float** dst, const std::vector<T>& src) {
  std::vector<float> f(src.begin(), src.end());
  return upload(c, dst, f);
}

}  // namespace

int upload_dm(Ctx& c, const HostMesh& m, DevMesh& d) {
  d.dim = m.dim;
  d.max_level = m.max_level;
  d.n = m.n_indep;
  d.n_hanging = m.n_hanging;
  d.n_slots = m.n_slots;
  d.n_colors = m.n_colors;
  d.side = 1 << m.max_level;
  // structured kernels address nodes with 32-bit offsets
  d.structured = m.uniform && m.node_order == 0 && m.n_hanging == 0 && m.n_indep < ((int64_t)1 << 31);
  int rc;
  for (int k = 0; k < kBrickClasses; ++k) {
    const BrickClass& h = m.cls[k];
    DevBrickClass& b = d.cls[k];
    b.B = h.B;
    b.count = h.count;
    b.npb = h.nodes_per_brick;
    b.nbnd = h.bnd_per_brick;
    b.slot_base = h.slot_base;
    if ((rc = upload(c, &b.table, h.table))) return rc;
    if ((rc = upload(c, &b.level, h.level))) return rc;
    std::vector<int16_t> r(h.rank.begin(), h.rank.end());
    if ((rc = upload(c, &b.rank, r))) return rc;
    if ((rc = upload(c, &b.anchor, h.anchor))) return rc;
    if (!h.abase.empty() && (rc = upload(c, &b.abase, h.abase))) return rc;
  }
  if ((rc = upload(c, &d.hang_par, m.hang_parents))) return rc;
  d.n_comb = (int64_t)m.comb_node.size();
  if ((rc = upload(c, &d.comb_node, m.comb_node))) return rc;
  if ((rc = upload(c, &d.comb_ptr, m.comb_ptr))) return rc;
  if ((rc = upload(c, &d.comb_ent, m.comb_ent))) return rc;
  if ((rc = upload(c, &d.color, m.color))) return rc;
  if ((rc = upload(c, &d.wall, m.wall))) return rc;
  return CHNS_OK;
}

namespace {

LevelView view(MgLevel& L) { return LevelView{&L.dm, L.phi64, L.phi32, L.slots}; }

// Host: dense inverse by Cholesky of A, of A + (scale/n) 1 1^T when
// regularise (singular pressure operator: the inverse then returns the
// mean-free solution for a right-hand side in the range).
int dense_inverse(std::vector<double>& A, int n, bool regularise) {
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, A[(size_t)i * n + i]);
  {
    const std::vector<double> A0(A);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = 0.5 * (A0[(size_t)i * n + j] + A0[(size_t)j * n + i]);
  }
  if (regularise)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) A[(size_t)i * n + j] += scale / n;
  std::vector<double> Lc((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= Lc[(size_t)j * n + k] * Lc[(size_t)j * n + k];
    if (!(d > 0.0)) return CHNS_EINVAL;
    d = std::sqrt(d);
    Lc[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= Lc[(size_t)i * n + k] * Lc[(size_t)j * n + k];
      Lc[(size_t)i * n + j] = v / d;
    }
  }
  // inverse column by column: L L^T x = e_j
  std::vector<double> inv((size_t)n * n), y(n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) {
      double v = (i == j) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= Lc[(size_t)i * n + k] * y[k];
      y[i] = v / Lc[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < n; ++k) v -= Lc[(size_t)k * n + i] * inv[(size_t)k * n + j];
      inv[(size_t)i * n + j] = v / Lc[(size_t)i * n + i];
    }
  }
  A.swap(inv);
  return CHNS_OK;
}

// The same inverse on the device for a coarsest level of at most
// kDenseDev nodes, in one wave: the host routine's steps in its order with
// fused multiply-adds off (division and square root are correctly rounded),
// so the inverse is the host's bit for bit without the round trip through
// host memory.  Cholesky: column by column, lane i forms the entry of row i;
// inverse: lane j forms column j by forward and back substitution.  A
// non-positive pivot makes the inverse NaN, and a solve that uses it stops
// on its non-finite residual.
constexpr int kDenseDev = 64;
__global__ __launch_bounds__(64) void k_dense_inverse(const double* __restrict__ A0, double* __restrict__ inv64,
                                                      float* __restrict__ inv32, int n, int regularise) {
#pragma clang fp contract(off)
  __shared__ double A[kDenseDev * kDenseDev], Lc[kDenseDev * kDenseDev], Y[kDenseDev * kDenseDev];
  const int t = threadIdx.x;
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = scale < A0[i * n + i] ? A0[i * n + i] : scale;
  for (int q = t; q < n * n; q += 64) {
    const int i = q / n, j = q % n;
    double a = 0.5 * (A0[i * n + j] + A0[j * n + i]);
    if (regularise) a += scale / n;
    A[q] = a;
    Lc[q] = 0.0;
  }
  wave_sync();
  bool bad = false;
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= Lc[j * n + k] * Lc[j * n + k];
    bad = bad || !(d > 0.0);
    d = sqrt(d);
    if (t == 0) Lc[j * n + j] = d;
    if (t > j && t < n) {
      double v = A[t * n + j];
      for (int k = 0; k < j; ++k) v -= Lc[t * n + k] * Lc[j * n + k];
      Lc[t * n + j] = v / d;
    }
    wave_sync();
  }
  if (t < n) {
    const int j = t;
    for (int i = 0; i < n; ++i) {
      double v = (i == j) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= Lc[i * n + k] * Y[k * kDenseDev + j];
      Y[i * kDenseDev + j] = v / Lc[i * n + i];
    }
    // column j of the inverse into A (row i at A[i * kDenseDev + j])
    for (int i = n - 1; i >= 0; --i) {
      double v = Y[i * kDenseDev + j];
      for (int k = i + 1; k < n; ++k) v -= Lc[k * n + i] * A[k * kDenseDev + j];
      A[i * kDenseDev + j] = v / Lc[i * n + i];
    }
  }
  wave_sync();
  for (int q = t; q < n * n; q += 64) {
    const int i = q / n, j = q % n;
    const double v = bad ? __builtin_nan("") : A[i * kDenseDev + j];
    inv64[q] = v;
    inv32[q] = (float)v;
  }
}

template <typename T>
struct Prec;
template <>
struct Prec<double> {
  static constexpr int P = CHNS_FP64;
  static double* v(MgLevel& L, int k) { return L.v64[k]; }
  static double* dinv(MgLevel& L) { return L.dinv64; }
  static const double* Pv(MgLevel& L) { return L.P_val64; }
  static const double* Rv(MgLevel& L) { return L.R_val64; }
  static const double* inv(MgLevel& L) { return L.inv64; }
  static double* fine_dinv(Multigrid& m) { return m.fine_dinv64; }
  static double* fine_t(Multigrid& m) { return m.fine_t64; }
};
template <>
struct Prec<float> {
  static constexpr int P = CHNS_FP32;
  static float* v(MgLevel& L, int k) { return L.v32[k]; }
  static float* dinv(MgLevel& L) { return L.dinv32; }
  static const float* Pv(MgLevel& L) { return L.P_val32; }
  static const float* Rv(MgLevel& L) { return L.R_val32; }
  static const float* inv(MgLevel& L) { return L.inv32; }
  static float* fine_dinv(Multigrid& m) { return m.fine_dinv32; }
  static float* fine_t(Multigrid& m) { return m.fine_t32; }
};

template <typename T>
int vcycle(Ctx& c, int k, const T* r, T* z, hipStream_t s);

// transfer y (+)= A x with L lanes per row; FP64 vectors read the FP32 copy
// of the weights when all of them are exact in FP32 (dyadic Q1 weights)
template <typename T, int L>
void transfer(const Multigrid& mg, const int32_t* ptr, const int32_t* col, const T* val, const float* val32,
              const T* x, T* y, int64_t rows, const T* yin, hipStream_t s) {
  const unsigned g = blocks(rows * L);
  if (sizeof(T) == 8 && mg.transfer32_exact)
    k_spmv_g<T, float, L><<<g, kT, 0, s>>>(ptr, col, val32, x, y, rows, yin);
  else
    k_spmv_g<T, T, L><<<g, kT, 0, s>>>(ptr, col, val, x, y, rows, yin);
}

// The rest of the cycle from stencil level k as one k_vcycle_tail launch,
// when every level from k down is a lexicographic stencil level and all of
// them fit in the tail's LDS (false: the per-level launches run instead).
template <typename T>
bool launch_tail(Ctx& c, int k, const T* r, T* z, hipStream_t s) {
  using PR = Prec<T>;
  Multigrid& mg = *c.mg;
  const int K = (int)mg.lv.size() - 1;
  if (k >= K || K - k > kTailLevels) return false;
  auto lex = [](const DevMesh& d) {
    const int64_t s1 = d.side + 1;
    return d.n == (d.dim == 3 ? s1 * s1 * s1 : s1 * s1);
  };
  TailArgs<T> a{};
  const int dim = mg.lv[k].dm.dim;
  const int64_t ns = dim == 3 ? 27 : 9;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off += (bytes + 15) / 16 * 16;
    return (int)std::min<int64_t>(o, kTailLds);
  };
  for (int j = k; j < K; ++j) {
    MgLevel& L = mg.lv[j];
    if (!L.S64 || !L.S32 || L.dm.dim != dim || !lex(L.dm) || mg.lv[j + 1].dm.side * 2 != L.dm.side ||
        L.dm.n > kTailLds)
      return false;
    const int64_t n = L.dm.n;
    TailLevel<T>& t = a.lv[j - k];
    t.S = L.S32;
    t.dinv = PR::dinv(L);
    t.z = z;
    t.side = L.dm.side;
    t.n = (int)n;
    t.oS = take(sizeof(float) * ns * n);
    t.od = take(sizeof(T) * n);
    t.orr = take(sizeof(T) * n);
    t.oz = take(sizeof(T) * n);
    t.ot = take(sizeof(T) * n);
    t.oz2 = take(sizeof(T) * n);
  }
  MgLevel& B = mg.lv[K];
  if (B.dm.dim != dim || !lex(B.dm) || B.dm.n > kTailLds) return false;
  a.nl = K - k;
  a.inv = PR::inv(B);
  a.sideK = B.dm.side;
  a.nK = (int)B.dm.n;
  a.oinv = take(sizeof(T) * B.dm.n * B.dm.n);
  a.orK = take(sizeof(T) * B.dm.n);
  a.ozK = take(sizeof(T) * B.dm.n);
  if (off > kTailLds) return false;
  auto seg = [&](const void* src, int dst, int64_t bytes) {
    TailSeg& g = a.seg[a.nseg++];
    g.src = static_cast<const char*>(src);
    g.dst = dst;
    g.bytes = (int)bytes;
    g.chunk0 = a.nchunk;
    a.nchunk += (int)(bytes / 16);
    return reinterpret_cast<uintptr_t>(src) % 16 == 0;
  };
  bool aligned = true;
  for (int l = 0; l < a.nl; ++l) {
    const TailLevel<T>& t = a.lv[l];
    aligned &= seg(t.S, t.oS, sizeof(float) * ns * t.n);
    aligned &= seg(t.dinv, t.od, sizeof(T) * t.n);
  }
  aligned &= seg(r, a.lv[0].orr, sizeof(T) * a.lv[0].n);
  aligned &= seg(a.inv, a.oinv, sizeof(T) * a.nK * a.nK);
  if (!aligned) return false;
  a.nu = mg.nu;
  a.w = (T)mg.omega;
  if (dim == 3) k_vcycle_tail<T, 3><<<1, kTailT, 0, s>>>(a);
  else k_vcycle_tail<T, 2><<<1, kTailT, 0, s>>>(a);
  return true;
}

// V-cycle from a uniform coarse level k > 0 with an assembled stencil: the
// same damped-Jacobi sweeps and transfers as the matrix-free levels, six
// launches per level (two-sweep pre-smoothing, A z, restriction,
// prolongation, two post-smoothing sweeps); the small levels at the bottom
// run fused in one launch
template <typename T>
int vcycle_stencil(Ctx& c, int k, const T* r, T* z, hipStream_t s) {
  using PR = Prec<T>;
  Multigrid& mg = *c.mg;
  MgLevel& L = mg.lv[k];
  if (launch_tail<T>(c, k, r, z, s)) {
    CHNS_HIP(hipGetLastError());
    return CHNS_OK;
  }
  MgLevel& C = mg.lv[k + 1];
  const int64_t n = L.dm.n;
  const int side = L.dm.side, dim = L.dm.dim;
  // the coarse operator's values are read in FP32 in both precisions (half
  // the stencil stream; the arithmetic stays in T, and the FP32-rounded
  // operator is a fixed symmetric matrix, so the cycle is still a fixed SPD
  // preconditioner)
  const float* S = L.S32;
  const T* dinv = PR::dinv(L);
  T* t = PR::v(L, 2);
  T* z2 = PR::v(L, 3);
  const T w = (T)mg.omega;
  const unsigned g = blocks(n);
  auto pre2 = [&]() {
    if (dim == 3) k_st_pre2<T, 3, float><<<g, kT, 0, s>>>(S, dinv, r, z, w, side, n);
    else k_st_pre2<T, 2, float><<<g, kT, 0, s>>>(S, dinv, r, z, w, side, n);
  };
  auto sweep = [&](const T* zi, T* zo) {
    if (dim == 3) k_st_sweep<T, 3, float><<<g, kT, 0, s>>>(S, dinv, r, zi, zo, w, side, n);
    else k_st_sweep<T, 2, float><<<g, kT, 0, s>>>(S, dinv, r, zi, zo, w, side, n);
  };
  // pre-smoothing: nu sweeps from a zero guess, result in z; t = A z
  if (mg.nu == 1) {
    if (dim == 3) k_st_pre1<T, 3, float><<<g, kT, 0, s>>>(S, dinv, r, z, t, w, side, n);
    else k_st_pre1<T, 2, float><<<g, kT, 0, s>>>(S, dinv, r, z, t, w, side, n);
  } else {
    pre2();
    for (int it = 2; it < mg.nu; ++it) {
      sweep(z, z2);
      k_copy_t<T><<<g, kT, 0, s>>>(z2, z, n);
    }
    if (dim == 3) k_st_apply<T, 3, float><<<g, kT, 0, s>>>(S, z, t, side, n);
    else k_st_apply<T, 2, float><<<g, kT, 0, s>>>(S, z, t, side, n);
  }
  T* rc_ = PR::v(C, 0);
  T* zc = PR::v(C, 1);
  if (dim == 3) k_restrict_s<T, 3><<<blocks(C.dm.n), kT, 0, s>>>(r, t, rc_, C.dm.side);
  else k_restrict_s<T, 2><<<blocks(C.dm.n), kT, 0, s>>>(r, t, rc_, C.dm.side);
  CHNS_HIP(hipGetLastError());
  int rc;
  if ((rc = vcycle<T>(c, k + 1, rc_, zc, s))) return rc;
  // post-smoothing: nu sweeps alternating between z and z2; for odd nu the
  // prolongation writes the corrected iterate to z2, so they end in z
  const bool odd = mg.nu % 2 == 1;
  T* cur = odd ? z2 : z;
  T* oth = odd ? z : z2;
  k_prolong_s<T><<<g, kT, 0, s>>>(zc, z, cur, C.dm.side, dim);
  for (int it = 0; it < mg.nu; ++it) {
    sweep(cur, oth);
    std::swap(cur, oth);
  }
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

// z = V(r) on level k (k = 0 is the context's mesh)
template <typename T>
int vcycle(Ctx& c, int k, const T* r, T* z, hipStream_t s) {
  Multigrid& mg = *c.mg;
  const int K = (int)mg.lv.size() - 1;
  using PR = Prec<T>;
  if (k == K) {
    MgLevel& L = mg.lv[k];
    k_dense<T><<<blocks(L.dm.n), kT, 0, s>>>(PR::inv(L), r, z, (int)L.dm.n);
    CHNS_HIP(hipGetLastError());
    return CHNS_OK;
  }
  const LevelView V = k == 0 ? fine_view(c) : view(mg.lv[k]);
  const int64_t n = V.dm->n;
  T* dinv = k == 0 ? PR::fine_dinv(mg) : PR::dinv(mg.lv[k]);
  T* t = k == 0 ? PR::fine_t(mg) : PR::v(mg.lv[k], 2);
  const T w = (T)mg.omega;
  const unsigned g = blocks(n);
  ApplyOut plain{};
  int rc;
  if (k > 0 && mg.lv[k].S64) return vcycle_stencil<T>(c, k, r, z, s);
  // sweeps fused into the apply (brick and combine write x + w D^-1 (r - A x)
  // into the other buffer), alternating between z and t so that the last
  // pre-smoothing sweep lands in z
  ApplyOut sm{};
  sm.sm_r = r;
  sm.sm_dinv = dinv;
  sm.sm_w = mg.omega;
  {
    T* cur = (mg.nu % 2 == 1) ? z : t;  // after nu - 1 sweeps the result is in z
    T* oth = cur == z ? t : z;
    k_jacobi0<T><<<g, kT, 0, s>>>(cur, r, dinv, w, n);
    for (int it = 1; it < mg.nu; ++it) {
      if ((rc = launch_apply_lv(c, V, CHNS_OP_PRESSURE, PR::P, cur, oth, s, sm))) return rc;
      std::swap(cur, oth);
    }
  }
  if ((rc = launch_apply_lv(c, V, CHNS_OP_PRESSURE, PR::P, z, t, s, plain))) return rc;
  MgLevel& C = mg.lv[k + 1];
  T* rc_ = PR::v(C, 0);
  T* zc = PR::v(C, 1);
  const bool structured = V.dm->structured && C.dm.structured;
  if (structured) {
    if (C.dm.dim == 3) k_restrict_s<T, 3><<<blocks(C.dm.n), kT, 0, s>>>(r, t, rc_, C.dm.side);
    else k_restrict_s<T, 2><<<blocks(C.dm.n), kT, 0, s>>>(r, t, rc_, C.dm.side);
  } else {
    k_resid<T><<<g, kT, 0, s>>>(r, t, n);
    transfer<T, 8>(mg, C.R_ptr, C.R_col, PR::Rv(C), C.R_val32, t, rc_, C.dm.n, nullptr, s);
  }
  CHNS_HIP(hipGetLastError());
  if ((rc = vcycle<T>(c, k + 1, rc_, zc, s))) return rc;
  // post-smoothing alternating between z and t; for odd nu the prolongation
  // writes the corrected iterate to t, so the sweeps end in z
  {
    const bool odd = mg.nu % 2 == 1;
    T* cur = odd ? t : z;
    T* oth = odd ? z : t;
    if (structured)
      k_prolong_s<T><<<g, kT, 0, s>>>(zc, z, cur, C.dm.side, C.dm.dim);
    else
      transfer<T, 4>(mg, C.P_ptr, C.P_col, PR::Pv(C), C.P_val32, zc, cur, n, z, s);
    for (int it = 0; it < mg.nu; ++it) {
      if ((rc = launch_apply_lv(c, V, CHNS_OP_PRESSURE, PR::P, cur, oth, s, sm))) return rc;
      std::swap(cur, oth);
    }
  }
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

}  // namespace

// Host: reference tables of the element-matrix Galerkin products (see the
// kernels above); bit d of a corner / Gauss point / child index is axis d.
void reference_tables(int dim, std::vector<double>& tg, std::vector<double>& tp, std::vector<double>& th,
                      std::vector<double>& tm, std::vector<double>& tmq, std::vector<double>& thm) {
  const int nc = 1 << dim, ne = nc * nc;
  const double g = 0.57735026918962576451;
  const double norm = dim == 3 ? 0.125 : 0.25;
  tg.assign((size_t)nc * ne, 0.0);
  for (int q = 0; q < nc; ++q) {
    double grad[8][3];
    for (int a = 0; a < nc; ++a)
      for (int d = 0; d < dim; ++d) {
        double v = norm * (((a >> d) & 1) ? 1.0 : -1.0);
        for (int d2 = 0; d2 < dim; ++d2)
          if (d2 != d) v *= 1.0 + (((a >> d2) & 1) ? 1.0 : -1.0) * (((q >> d2) & 1) ? g : -g);
        grad[a][d] = v;
      }
    for (int a = 0; a < nc; ++a)
      for (int b = 0; b < nc; ++b) {
        double v = 0.0;
        for (int d = 0; d < dim; ++d) v += grad[a][d] * grad[b][d];
        tg[(size_t)q * ne + a * nc + b] = v;
      }
  }
  // P_c(b, A): fine position c_d + b_d in {0, 1, 2} against coarse corner A_d
  tp.assign((size_t)nc * ne, 0.0);
  for (int c = 0; c < nc; ++c)
    for (int b = 0; b < nc; ++b)
      for (int A = 0; A < nc; ++A) {
        double w = 1.0;
        for (int d = 0; d < dim; ++d) {
          const int f = ((c >> d) & 1) + ((b >> d) & 1), ad = (A >> d) & 1;
          w *= f == 1 ? 0.5 : ((f == 0) == (ad == 0) ? 1.0 : 0.0);
        }
        tp[((size_t)c * nc + b) * nc + A] = w;
      }
  // reference mass: N_a N_b at each Gauss point (N = prod (1 +- xi) / 2)
  // and its sum over them
  tm.assign((size_t)ne, 0.0);
  tmq.assign((size_t)nc * ne, 0.0);
  for (int q = 0; q < nc; ++q)
    for (int a = 0; a < nc; ++a)
      for (int b = 0; b < nc; ++b) {
        double na = 1.0, nb = 1.0;
        for (int d = 0; d < dim; ++d) {
          const double xq = ((q >> d) & 1) ? g : -g;
          na *= 0.5 * (1.0 + (((a >> d) & 1) ? 1.0 : -1.0) * xq);
          nb *= 0.5 * (1.0 + (((b >> d) & 1) ? 1.0 : -1.0) * xq);
        }
        tm[(size_t)a * nc + b] += na * nb;
        tmq[(size_t)q * ne + a * nc + b] = na * nb;
      }
  // Galerkin products P_c^T T_q P_c of the per-point stiffness and mass
  auto galerkin = [&](const std::vector<double>& t, std::vector<double>& out) {
    out.assign((size_t)ne * ne, 0.0);
    for (int c = 0; c < nc; ++c)
      for (int q = 0; q < nc; ++q)
        for (int A = 0; A < nc; ++A)
          for (int B = 0; B < nc; ++B) {
            double v = 0.0;
            for (int a = 0; a < nc; ++a)
              for (int b = 0; b < nc; ++b)
                v += tp[((size_t)c * nc + a) * nc + A] * t[(size_t)q * ne + a * nc + b] *
                     tp[((size_t)c * nc + b) * nc + B];
            out[(size_t)(c * nc + q) * ne + A * nc + B] = v;
          }
  };
  galerkin(tg, th);
  galerkin(tmq, thm);
}

int mg_build(Ctx& c) {
  if (c.mg) return CHNS_OK;
  const HostMesh& f = *c.host;
  // a carved octree keeps its domain only down to the carve level
  const int coarsest = std::max(1, f.carve_level);
  auto* mg = new Multigrid();
  mg->lv.resize(1);
  std::string msg;
  const HostMesh* finer = &f;
  for (int k = f.max_level - 1; k >= coarsest; --k) {
    MgLevel L;
    std::vector<int8_t> lev;
    std::vector<int32_t> anc;
    truncate_leaves(*finer, k, lev, anc);
    int rc = build_host_mesh_from_leaves(f.dim, k, lev, anc, L.host, msg, &f);
    if (rc) {
      delete mg;
      set_error("multigrid level: " + msg);
      return rc;
    }
    mg->lv.push_back(std::move(L));
    finer = &mg->lv.back().host;
  }
  if (mg->lv.size() < 2) {
    delete mg;
    set_error("mesh too coarse for multigrid (needs max_level >= 2)");
    return CHNS_EINVAL;
  }
  int rc;
  for (size_t k = 1; k < mg->lv.size(); ++k) {
    MgLevel& L = mg->lv[k];
    const HostMesh& fine = k == 1 ? f : mg->lv[k - 1].host;
    Transfer t;
    if ((rc = build_transfer(fine, L.host, t, msg))) {
      delete mg;
      set_error("multigrid transfer: " + msg);
      return rc;
    }
    if ((rc = upload_dm(c, L.host, L.dm))) goto fail;
    if (k == 1) mg->transfer32_exact = true;
    for (const std::vector<double>* vals : {&t.P_val, &t.R_val})
      for (double v : *vals)
        if ((double)(float)v != v) mg->transfer32_exact = false;
    L.P_rows = fine.n_indep;
    if ((rc = upload(c, &L.P_ptr, t.P_ptr)) || (rc = upload(c, &L.P_col, t.P_col)) ||
        (rc = upload(c, &L.P_val64, t.P_val)) || (rc = upload_as_float(c, &L.P_val32, t.P_val)) ||
        (rc = upload(c, &L.R_ptr, t.R_ptr)) || (rc = upload(c, &L.R_col, t.R_col)) ||
        (rc = upload(c, &L.R_val64, t.R_val)) || (rc = upload_as_float(c, &L.R_val32, t.R_val)) ||
        (rc = upload(c, &L.I_ptr, t.I_ptr)) || (rc = upload(c, &L.I_col, t.I_col)) ||
        (rc = upload(c, &L.I_val, t.I_val)))
      goto fail;
    {
      const int64_t n = L.dm.n;
      L.phi64 = (double*)c.dalloc(sizeof(double) * n);
      L.phi32 = (float*)c.dalloc(sizeof(float) * n);
      L.slots = c.dalloc(sizeof(double) * (size_t)(L.dm.n_slots > 0 ? L.dm.n_slots : 1) * 3);
      L.dinv64 = (double*)c.dalloc(sizeof(double) * n);
      L.dinv32 = (float*)c.dalloc(sizeof(float) * n);
      for (int j = 0; j < 4; ++j) {
        L.v64[j] = (double*)c.dalloc(sizeof(double) * n);
        L.v32[j] = (float*)c.dalloc(sizeof(float) * n);
        if (!L.v64[j] || !L.v32[j]) {
          rc = CHNS_ENOMEM;
          goto fail;
        }
      }
      if (!L.phi64 || !L.phi32 || !L.slots || !L.dinv64 || !L.dinv32) {
        rc = CHNS_ENOMEM;
        goto fail;
      }
    }
  }
  // stencils and element matrices: every uniform level above the coarsest
  // whose next coarser level is uniform (stencil V-cycle), and the uniform
  // coarsest level when the level above it is uniform (dense matrix from
  // the Galerkin product)
  {
    const size_t K = mg->lv.size() - 1;
    for (size_t k = 1; k <= K; ++k) {
      MgLevel& L = mg->lv[k];
      if (!L.dm.structured) continue;
      const bool finer_st = k == 1 ? c.dm.structured : mg->lv[k - 1].dm.structured;
      const bool vcyc = k < K && mg->lv[k + 1].dm.structured;
      if (!vcyc && !(k == K && finer_st)) continue;
      const int64_t ns = (L.dm.dim == 3 ? 27 : 9) * L.dm.n;
      const int64_t ne = (int64_t)1 << (L.dm.dim * L.host.max_level);
      L.S64 = (double*)c.dalloc(sizeof(double) * ns);
      L.E64 = (double*)c.dalloc(sizeof(double) * ne * (L.dm.dim == 3 ? 64 : 16));
      if (vcyc) L.S32 = (float*)c.dalloc(sizeof(float) * ns);
      if (!L.S64 || !L.E64 || (vcyc && !L.S32)) {
        rc = CHNS_ENOMEM;
        goto fail;
      }
    }
    std::vector<double> tg, tp, th, tm, tmq, thm;
    reference_tables(c.dm.dim, tg, tp, th, tm, tmq, thm);
    if ((rc = upload(c, &mg->tab_G, tg)) || (rc = upload(c, &mg->tab_P, tp)) || (rc = upload(c, &mg->tab_M, tm)) ||
        (rc = upload(c, &mg->tab_Mq, tmq)))
      goto fail;
    if (c.dm.structured && mg->lv[1].E64) {
      if ((rc = upload(c, &mg->tab_H, th)) || (rc = upload(c, &mg->tab_Hm, thm))) goto fail;
      const int64_t ncoarse = (int64_t)1 << (c.dm.dim * (c.dm.max_level - 1));
      mg->diag_part = (double*)c.dalloc(sizeof(double) * (size_t)ncoarse * (c.dm.dim == 3 ? 27 : 9));
      if (!mg->diag_part) {
        rc = CHNS_ENOMEM;
        goto fail;
      }
    }
  }
  {
    MgLevel& B = mg->lv.back();
    const int64_t n = B.dm.n;
    B.dense = (double*)c.dalloc(sizeof(double) * n * n);
    B.inv64 = (double*)c.dalloc(sizeof(double) * n * n);
    B.inv32 = (float*)c.dalloc(sizeof(float) * n * n);
    const int64_t nf = c.dm.n;
    mg->fine_dinv64 = (double*)c.dalloc(sizeof(double) * nf);
    mg->fine_dinv32 = (float*)c.dalloc(sizeof(float) * nf);
    mg->fine_t64 = (double*)c.dalloc(sizeof(double) * nf);
    mg->fine_t32 = (float*)c.dalloc(sizeof(float) * nf);
    if (!B.dense || !B.inv64 || !B.inv32 || !mg->fine_dinv64 || !mg->fine_dinv32 || !mg->fine_t64 ||
        !mg->fine_t32) {
      rc = CHNS_ENOMEM;
      goto fail;
    }
  }
  c.mg = mg;
  return CHNS_OK;
fail:
  delete mg;
  return rc;
}

// Per phase field: inject phi~ down the levels, exact diagonals, coarse
// operator columns (device part captured once into a graph), then the
// regularised inverse of the coarsest operator on the host.
int mg_setup(Ctx& c, hipStream_t s) {
  Multigrid& mg = *c.mg;
  int rc;
  // smoothing per operator: the pressure Poisson cycle (CG) runs one
  // damped-Jacobi sweep each way with omega 0.9 (fewer fine-level applies
  // per iteration outweigh the extra iteration); the shifted and momentum
  // cycles inside GMRES keep two sweeps with omega 0.6
  const bool pressure = c.pp_kind == 0 && c.pp_shift == 0.0;
  mg.nu = pressure ? 1 : 2;
  mg.omega = pressure ? 0.9 : 0.6;
  for (int k = 6; k < 8; ++k) {
    if (!c.w64[k]) c.w64[k] = (double*)c.dalloc(sizeof(double) * c.dm.n * 3);
    if (!c.w32[k]) c.w32[k] = (float*)c.dalloc(sizeof(float) * c.dm.n * 3);
    if (!c.w64[k] || !c.w32[k]) return CHNS_ENOMEM;
  }
  MgLevel& B = mg.lv.back();
  const int n = (int)B.dm.n;
  auto device_part = [&](hipStream_t st) -> int {
    int e;
    const double al = (c.prm.rho_plus - c.prm.rho_minus) / (2.0 * c.prm.rho_plus);
    const double be = (c.prm.rho_plus + c.prm.rho_minus) / (2.0 * c.prm.rho_plus);
    const int dim = c.dm.dim;
    QCoef cf{al, be, 0.0, c.pp_shift, 0};
    if (c.pp_kind == 1) {
      // eta/(2 Re) on the stiffness, rho/dt on the mass
      const double ga = (c.prm.eta_plus - c.prm.eta_minus) / (2.0 * c.prm.eta_plus);
      const double xi = (c.prm.eta_plus + c.prm.eta_minus) / (2.0 * c.prm.eta_plus);
      cf = QCoef{ga / (2.0 * c.prm.Re), xi / (2.0 * c.prm.Re), al / c.prm.dt, be / c.prm.dt, 1};
    }
    const bool varm = cf.ma != 0.0;
    // (h/2)^(d-2) and det J = (h/2)^d of a uniform level with s cells per edge
    auto lscale = [&](int s) { return dim == 3 ? 0.5 / s : 1.0; };
    auto mscale = [&](int s) { return std::pow(0.5 / s, dim); };
    if (mg.tab_H) {
      // uniform fine level: inverse diagonal straight from the phase field,
      // first coarse level's element matrices as Galerkin products
      const int64_t ncoarse = (int64_t)1 << (dim * (c.dm.max_level - 1));
      const unsigned gl = (unsigned)((ncoarse + kGalPerWave - 1) / kGalPerWave);
      const int sf = c.dm.side;
      // k_gal_phi takes element coordinates by shifts: a power-of-two side
      if (sf < 2 || (sf & (sf - 1)) != 0 || ncoarse != std::pow((double)(sf / 2), dim)) {
        set_error("multigrid: uniform fine level with a side that is not a power of two");
        return CHNS_EINVAL;
      }
      const double mc = cf.mb * mscale(sf / 2);
      const double fm = mscale(sf);
      if (dim == 3) {
        if (varm)
          k_gal_phi<3, true><<<gl, 64, 0, st>>>(c.phi64, sf, mg.tab_H, cf, lscale(sf), mg.lv[1].E64, ncoarse,
                                                mg.tab_M, mc, mg.tab_Hm, mscale(sf), mg.tab_G, mg.tab_Mq, fm,
                                                mg.diag_part);
        else
          k_gal_phi<3, false><<<gl, 64, 0, st>>>(c.phi64, sf, mg.tab_H, cf, lscale(sf), mg.lv[1].E64, ncoarse,
                                                 mg.tab_M, mc, mg.tab_Hm, mscale(sf), mg.tab_G, mg.tab_Mq, fm,
                                                 mg.diag_part);
        k_diag_gather<3><<<blocks(c.dm.n), kT, 0, st>>>(mg.diag_part, sf / 2, mg.fine_dinv64, mg.fine_dinv32);
      } else {
        if (varm)
          k_gal_phi<2, true><<<gl, 64, 0, st>>>(c.phi64, sf, mg.tab_H, cf, lscale(sf), mg.lv[1].E64, ncoarse,
                                                mg.tab_M, mc, mg.tab_Hm, mscale(sf), mg.tab_G, mg.tab_Mq, fm,
                                                mg.diag_part);
        else
          k_gal_phi<2, false><<<gl, 64, 0, st>>>(c.phi64, sf, mg.tab_H, cf, lscale(sf), mg.lv[1].E64, ncoarse,
                                                 mg.tab_M, mc, mg.tab_Hm, mscale(sf), mg.tab_G, mg.tab_Mq, fm,
                                                 mg.diag_part);
        k_diag_gather<2><<<blocks(c.dm.n), kT, 0, st>>>(mg.diag_part, sf / 2, mg.fine_dinv64, mg.fine_dinv32);
      }
      CHNS_HIP(hipGetLastError());
    } else {
      if ((e = launch_diagonal_lv(c, fine_view(c), CHNS_OP_PRESSURE, CHNS_FP64, mg.fine_dinv64, true, c.w64[6],
                                  c.w64[7], st)))
        return e;
      if ((e = launch_diagonal_lv(c, fine_view(c), CHNS_OP_PRESSURE, CHNS_FP32, mg.fine_dinv32, true, c.w32[6],
                                  c.w32[7], st)))
        return e;
    }
    const double* phi_f = c.phi64;
    for (size_t k = 1; k < mg.lv.size(); ++k) {
      MgLevel& L = mg.lv[k];
      const int64_t nk = L.dm.n;
      const DevMesh& F = k == 1 ? c.dm : mg.lv[k - 1].dm;
      // element matrices: Galerkin products from the level above when it has
      // them (done there), else rediscretised from the injected field; a
      // Galerkin level (and every level below it) needs no phase field
      const bool from_above = L.E64 && (k == 1 ? mg.tab_H != nullptr : mg.lv[k - 1].E64 != nullptr);
      if (!from_above) {
        if (F.structured && L.dm.structured)
          k_inject_s<<<blocks(nk), kT, 0, st>>>(phi_f, L.phi64, L.dm.side, L.dm.dim);
        else
          k_spmv<double, double><<<blocks(nk), kT, 0, st>>>(L.I_ptr, L.I_col, L.I_val, phi_f, L.phi64, nk, 0);
        k_phase32<<<blocks(nk), kT, 0, st>>>(L.phi64, L.phi32, nk);
        CHNS_HIP(hipGetLastError());
        phi_f = L.phi64;
      }
      if (L.E64) {
        const unsigned ne = (unsigned)((int64_t)1 << (dim * L.host.max_level));
        if (!from_above) {
          if (dim == 3)
            k_el_rediscr<3><<<ne, 64, 0, st>>>(L.phi64, L.dm.side, mg.tab_G, cf, lscale(L.dm.side), L.E64,
                                               mg.tab_Mq, mscale(L.dm.side));
          else
            k_el_rediscr<2><<<ne, 64, 0, st>>>(L.phi64, L.dm.side, mg.tab_G, cf, lscale(L.dm.side), L.E64,
                                               mg.tab_Mq, mscale(L.dm.side));
        }
        const bool last = k + 1 == mg.lv.size();
        double* d64 = last ? nullptr : L.dinv64;
        float* d32 = last ? nullptr : L.dinv32;
        // the cycle reads the stencils in FP32; the FP64 copy only feeds the
        // coarsest level's dense matrix
        double* s64 = last ? L.S64 : nullptr;
        if (dim == 3) k_el_stencil<3><<<blocks(nk), kT, 0, st>>>(L.E64, L.dm.side, s64, L.S32, d64, d32);
        else k_el_stencil<2><<<blocks(nk), kT, 0, st>>>(L.E64, L.dm.side, s64, L.S32, d64, d32);
        if (!last && mg.lv[k + 1].E64) {
          const unsigned nc = ne >> dim;
          if (dim == 3) k_gal_elem<3><<<nc, 64, 0, st>>>(L.E64, L.dm.side, mg.tab_P, mg.lv[k + 1].E64);
          else k_gal_elem<2><<<nc, 64, 0, st>>>(L.E64, L.dm.side, mg.tab_P, mg.lv[k + 1].E64);
        }
        CHNS_HIP(hipGetLastError());
      } else if (k + 1 < mg.lv.size()) {
        if ((e = launch_diagonal_lv(c, view(L), CHNS_OP_PRESSURE, CHNS_FP64, L.dinv64, true, L.v64[0], L.v64[3],
                                    st)))
          return e;
        if ((e = launch_diagonal_lv(c, view(L), CHNS_OP_PRESSURE, CHNS_FP32, L.dinv32, true, L.v32[0], L.v32[3],
                                    st)))
          return e;
      }
    }
    if (B.S64) {
      if (B.dm.dim == 3) k_stencil_dense<3><<<blocks(n), kT, 0, st>>>(B.S64, B.dm.side, B.dense);
      else k_stencil_dense<2><<<blocks(n), kT, 0, st>>>(B.S64, B.dm.side, B.dense);
      CHNS_HIP(hipGetLastError());
      return CHNS_OK;
    }
    ApplyOut plain{};
    for (int j = 0; j < n; ++j) {
      k_unit<<<blocks(n), kT, 0, st>>>(B.v64[0], j, n);
      if ((e = launch_apply_lv(c, view(B), CHNS_OP_PRESSURE, CHNS_FP64, B.v64[0], B.v64[3], st, plain))) return e;
      k_copy_col<<<blocks(n), kT, 0, st>>>(B.v64[3], B.dense, j, n);
    }
    CHNS_HIP(hipGetLastError());
    return CHNS_OK;
  };
  // the captured kernels carry the coefficients: one graph per shift value
  // and one for the scalar momentum operator
  hipGraphExec_t* exec = &mg.setup_exec;
  if (c.pp_kind == 1) {
    exec = &mg.mom_setup_exec;
  } else if (c.pp_shift != 0.0) {
    exec = nullptr;
    for (auto& e : mg.shifted_setups)
      if (e.first == c.pp_shift) exec = &e.second;
    if (!exec) {
      mg.shifted_setups.push_back({c.pp_shift, nullptr});
      exec = &mg.shifted_setups.back().second;
    }
  }
  if ((rc = run_captured(c, exec, s, device_part))) return rc;
  // a shifted operator or one with a mass term is definite: no rank-one
  // regularisation
  const bool regularise = c.pp_shift == 0.0 && c.pp_kind == 0;
  if (n <= kDenseDev) {
    k_dense_inverse<<<1, 64, 0, s>>>(B.dense, B.inv64, B.inv32, n, regularise ? 1 : 0);
  } else {
    std::vector<double> A((size_t)n * n);
    CHNS_HIP(hipMemcpyAsync(A.data(), B.dense, sizeof(double) * A.size(), hipMemcpyDeviceToHost, s));
    CHNS_HIP(hipStreamSynchronize(s));
    if ((rc = dense_inverse(A, n, regularise))) {
      set_error("coarsest multigrid operator is not positive semi-definite");
      return rc;
    }
    CHNS_HIP(hipMemcpy(B.inv64, A.data(), sizeof(double) * A.size(), hipMemcpyHostToDevice));
    k_to32<<<blocks((int64_t)n * n), kT, 0, s>>>(B.inv64, B.inv32, (int64_t)n * n);
  }
  CHNS_HIP(hipGetLastError());
  mg.setup_valid = true;
  return CHNS_OK;
}

int mg_vcycle64(Ctx& c, const double* r, double* z, hipStream_t s) { return vcycle<double>(c, 0, r, z, s); }

int interp_apply(const int32_t* ptr, const int32_t* col, const double* val, int64_t rows, int64_t cols, int nf,
                 const double* x, double* y, hipStream_t s) {
  for (int f = 0; f < nf; ++f)
    k_spmv_g<double, double, 4><<<blocks(rows * 4), kT, 0, s>>>(ptr, col, val, x + f * cols, y + f * rows, rows,
                                                                nullptr);
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}
int mg_vcycle32(Ctx& c, const float* r, float* z, hipStream_t s) { return vcycle<float>(c, 0, r, z, s); }

}  // namespace chns
