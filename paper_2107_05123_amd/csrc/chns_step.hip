// One projection time step of the Cahn-Hilliard Navier-Stokes system on the
// GPU, and the solvers it needs beyond the pressure CG:
//   * restarted right-preconditioned GMRES for the non-symmetric Newton
//     Jacobian of the Cahn-Hilliard system (Def. 6) and the VMS velocity
//     prediction (Def. 3); classical Gram-Schmidt applied twice, with the
//     Hessenberg matrix, the Givens rotations and the convergence test kept
//     on the device, so one Arnoldi step is a fixed kernel sequence that is
//     replayed from a HIP graph;
//   * Newton's method for the Cahn-Hilliard block (host loop over device
//     residual norms);
//   * the block iteration of the projection step: CH -> velocity prediction
//     -> pressure Poisson (Def. 4) -> velocity update (Def. 5), twice per
//     step (the paper's flowchart of the scheme).
// Every reduction is a fixed-order tree, so a step is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "chns_internal.h"

namespace chns {

constexpr int kGmMax = 128;  // largest GMRES restart length
constexpr int kT = 256;
constexpr int kMaxBlocks = 512;

// GMRES state on the device.  H is column-major, column j holds the rotated
// (upper-triangular) column of the Hessenberg matrix.
struct GmDev {
  int j, m, done, conv;  // completed Arnoldi steps, restart length, flags
  double tol, hinv, ww, beta;
  double g[kGmMax + 1], cs[kGmMax], sn[kGmMax], y[kGmMax];
  double h1[kGmMax + 1], h2[kGmMax + 1];
  double H[(kGmMax + 1) * kGmMax];
};

// GPC_SCHUR: block lower-triangular preconditioner of the Cahn-Hilliard
// Jacobian with a multigrid Schur-complement approximation (pcd = lumped mass)
// GPC_VPMG: one multigrid V-cycle of the scalar momentum operator per
// velocity component (interior rows), identity on the wall rows.
enum GmPc { GPC_NONE = 0, GPC_JACOBI = 1, GPC_BLOCK2 = 2, GPC_SCHUR = 3, GPC_VPMG = 4 };

struct Stepper {
  int64_t n = 0, nv = 0;  // nodes, longest vector (max(2, dim) * n)
  int m = 0;              // restart length the basis is sized for
  double* V = nullptr;    // (m + 1) * nv
  double* z = nullptr;
  double* w = nullptr;
  double* part = nullptr;  // (kGmMax + 1) * kMaxBlocks
  double* red = nullptr;   // reduction results (device)
  GmDev* gd = nullptr;
  GmDev* gd_host = nullptr;  // pinned
  double* red_host = nullptr;  // pinned
  hipEvent_t ev[4] = {};
  struct Graph {
    int op, pc;
    const void* pcdata;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  // time-step arrays
  double *X = nullptr, *R = nullptr, *dX = nullptr, *rhs = nullptr;
  double *uhat = nullptr, *ut = nullptr, *unew = nullptr, *v = nullptr, *pnew = nullptr;
  double *phit = nullptr, *mut = nullptr, *ycoord = nullptr, *tmp = nullptr, *zero = nullptr;
  double *blk = nullptr, *binv = nullptr, *dvp = nullptr, *dvu = nullptr, *dm = nullptr;
  // Cahn-Hilliard Schur-complement preconditioner: lumped mass, work vectors
  double *mL = nullptr, *pin = nullptr, *pout = nullptr, *pt1 = nullptr, *pt2 = nullptr, *pz = nullptr,
         *pj = nullptr;
  double *dMinv = nullptr, *cx = nullptr, *cr = nullptr, *cd = nullptr;  // Chebyshev solve with M
  double* vmask = nullptr;  // momentum multigrid preconditioner: masked input component
  double* fch = nullptr;    // Cahn-Hilliard body-force vector [-M f_phi; M f_mu]
  double sc_scale = 0.0;  // dt / b of the Schur approximation
  double m_lmax = 0.0;    // Gershgorin bound of eig(D_M^-1 M)
};

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// block of kT threads: fixed-order sum, result valid in thread 0
__device__ double bsum(double v, double* sh) {
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

inline unsigned blocks_for(int64_t n) {
  int64_t g = (n + kT - 1) / kT;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, kMaxBlocks));
}
// elementwise kernels (no reduction, so the grid does not change any result):
// enough blocks to fill every SIMD with waves, which keeps their streams'
// loads in flight
inline unsigned blocks_ew(int64_t n) {
  int64_t g = (n + kT - 1) / kT;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

#define GRID_LOOP(i, n) for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < (n); i += (int64_t)gridDim.x * kT)

// ------------------------------------------------------------ reductions
__global__ __launch_bounds__(kT) void k_dot_part(const double* a, const double* b, int64_t n, double* part) {
  __shared__ double sh[4];
  double v = 0.0;
  GRID_LOOP(i, n) v += a[i] * (b ? b[i] : 1.0);
  v = bsum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}
__global__ __launch_bounds__(kT) void k_sum_part(const double* part, int np, double* out) {
  __shared__ double sh[4];
  double v = 0.0;
  for (int k = threadIdx.x; k < np; k += kT) v += part[k];
  v = bsum(v, sh);
  if (threadIdx.x == 0) *out = v;
}

// ------------------------------------------------------- vector kernels
__global__ void k_axpby(double* out, double a, const double* x, double b, const double* y, int64_t n) {
  GRID_LOOP(i, n) out[i] = a * x[i] + b * y[i];
}
__global__ void k_scal(double* out, double a, const double* x, int64_t n) { GRID_LOOP(i, n) out[i] = a * x[i]; }
__global__ void k_fill0(double* x, int64_t n) { GRID_LOOP(i, n) x[i] = 0.0; }
__global__ void k_fill1(double* x, int64_t n) { GRID_LOOP(i, n) x[i] = 1.0; }
__global__ void k_add(double* x, const double* d, int64_t n) { GRID_LOOP(i, n) x[i] += d[i]; }

// inverse of the 2 x 2 node blocks [a b; c d] (row-major field blocks)
__global__ void k_inv2(const double* blk, double* inv, int64_t n) {
  GRID_LOOP(i, n) {
    const double a = blk[i], b = blk[n + i], c = blk[2 * n + i], d = blk[3 * n + i];
    const double det = a * d - b * c;
    const double r = det != 0.0 ? 1.0 / det : 0.0;
    inv[i] = d * r;
    inv[n + i] = -b * r;
    inv[2 * n + i] = -c * r;
    inv[3 * n + i] = a * r;
  }
}

// ---------------------------------------------------------------- GMRES
// z = M^-1 V_j
__global__ void k_gm_pc(const double* V, int64_t nv, int64_t n, double* z, const GmDev* gd, int pc,
                        const double* pcd) {
  if (gd->done) return;
  const double* v = V + (int64_t)gd->j * nv;
  if (pc == GPC_BLOCK2) {
    GRID_LOOP(i, n) {
      const double a = v[i], b = v[n + i];
      z[i] = pcd[i] * a + pcd[n + i] * b;
      z[n + i] = pcd[2 * n + i] * a + pcd[3 * n + i] * b;
    }
  } else if (pc == GPC_JACOBI) {
    GRID_LOOP(i, nv) z[i] = pcd[i] * v[i];
  } else {
    GRID_LOOP(i, nv) z[i] = v[i];
  }
}

// partial dots V_k . w for k <= j, four basis vectors per pass
__global__ __launch_bounds__(kT) void k_gm_multidot(const double* V, int64_t nv, const double* w, const GmDev* gd,
                                                    double* part) {
  __shared__ double sh[4][4];
  if (gd->done) return;
  const int j = gd->j;
  const int64_t i0 = (int64_t)blockIdx.x * kT + threadIdx.x, st = (int64_t)gridDim.x * kT;
  for (int k0 = 0; k0 <= j; k0 += 4) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    const int nk = min(4, j + 1 - k0);
    // two elements per trip, every load of the trip in flight together; each
    // thread still adds its elements in grid-stride order
    int64_t i = i0;
    for (; i + st < nv; i += 2 * st) {
      const double wa = w[i], wb = w[i + st];
      double va[4], vb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nk) {
          va[q] = V[(int64_t)(k0 + q) * nv + i];
          vb[q] = V[(int64_t)(k0 + q) * nv + i + st];
        }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nk) {
          a[q] += va[q] * wa;
          a[q] += vb[q] * wb;
        }
    }
    if (i < nv) {
      const double wi = w[i];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nk) a[q] += V[(int64_t)(k0 + q) * nv + i] * wi;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double t = wsum(a[q]);
      if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x < nk)
      part[(int64_t)(k0 + threadIdx.x) * gridDim.x + blockIdx.x] =
          (sh[threadIdx.x][0] + sh[threadIdx.x][1]) + (sh[threadIdx.x][2] + sh[threadIdx.x][3]);
    __syncthreads();
  }
}
// h[k] = sum of the partials of dot k (one block per k)
__global__ __launch_bounds__(kT) void k_gm_fin(const double* part, int np, GmDev* gd, int which) {
  __shared__ double sh[4];
  if (gd->done) return;
  const int k = blockIdx.x;
  if (k > gd->j) return;
  double v = 0.0;
  for (int t = threadIdx.x; t < np; t += kT) v += part[(int64_t)k * np + t];
  v = bsum(v, sh);
  if (threadIdx.x == 0) (which == 1 ? gd->h1 : gd->h2)[k] = v;
}
// w -= sum_k h[k] V_k; with `norm`, partial w.w into part[block].  The
// coefficients are staged in LDS and four basis loads issued per trip (the
// subtractions keep the order k = 0, 1, ..., j).
__global__ __launch_bounds__(kT) void k_gm_orth(const double* V, int64_t nv, double* w, const GmDev* gd, int which,
                                                double* part) {
  __shared__ double sh[4];
  __shared__ double hs[kGmMax + 1];
  if (gd->done) return;
  const int j = gd->j;
  const double* h = which == 1 ? gd->h1 : gd->h2;
  if (threadIdx.x <= j) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  double ww = 0.0;
  GRID_LOOP(i, nv) {
    double t = w[i];
    int k = 0;
    for (; k + 3 <= j; k += 4) {
      const double v0 = V[(int64_t)k * nv + i], v1 = V[(int64_t)(k + 1) * nv + i];
      const double v2 = V[(int64_t)(k + 2) * nv + i], v3 = V[(int64_t)(k + 3) * nv + i];
      t -= hs[k] * v0;
      t -= hs[k + 1] * v1;
      t -= hs[k + 2] * v2;
      t -= hs[k + 3] * v3;
    }
    for (; k <= j; ++k) t -= hs[k] * V[(int64_t)k * nv + i];
    w[i] = t;
    ww += t * t;
  }
  if (which == 2) {
    ww = bsum(ww, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = ww;
  }
}
// new Hessenberg column, Givens rotations, residual estimate, flags
__global__ __launch_bounds__(kT) void k_gm_givens(const double* part, int np, GmDev* gd) {
  __shared__ double sh[4];
  if (gd->done) return;
  double v = 0.0;
  for (int t = threadIdx.x; t < np; t += kT) v += part[t];
  v = bsum(v, sh);
  if (threadIdx.x != 0) return;
  const int j = gd->j, M1 = gd->m + 1;
  const double hn = sqrt(v);
  double* col = gd->H + (int64_t)j * M1;
  for (int k = 0; k <= j; ++k) col[k] = gd->h1[k] + gd->h2[k];
  col[j + 1] = hn;
  for (int k = 0; k < j; ++k) {
    const double a = col[k], b = col[k + 1];
    col[k] = gd->cs[k] * a + gd->sn[k] * b;
    col[k + 1] = -gd->sn[k] * a + gd->cs[k] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double r = hypot(a, b);
  const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? b / r : 0.0;
  gd->cs[j] = c;
  gd->sn[j] = s;
  col[j] = r;
  col[j + 1] = 0.0;
  gd->g[j + 1] = -s * gd->g[j];
  gd->g[j] = c * gd->g[j];
  gd->j = j + 1;
  gd->hinv = hn > 0.0 ? 1.0 / hn : 0.0;
  if (fabs(gd->g[j + 1]) <= gd->tol) {
    gd->conv = 1;
    gd->done = 1;
  }
  if (j + 1 >= gd->m || !(hn > 0.0)) gd->done = 1;
}
// V_j = w / |w| (j already advanced)
__global__ void k_gm_scale(double* V, int64_t nv, const double* w, const GmDev* gd) {
  if (gd->done) return;
  double* out = V + (int64_t)gd->j * nv;
  const double s = gd->hinv;
  GRID_LOOP(i, nv) out[i] = w[i] * s;
}
// cycle start: w = b - A x already in w, partial w.w in part
__global__ __launch_bounds__(kT) void k_gm_start(const double* part, int np, GmDev* gd, double tol, int m) {
  __shared__ double sh[4];
  double v = 0.0;
  for (int t = threadIdx.x; t < np; t += kT) v += part[t];
  v = bsum(v, sh);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(v);
  gd->beta = beta;
  gd->tol = tol;
  gd->m = m;
  gd->j = 0;
  gd->g[0] = beta;
  for (int k = 1; k <= m; ++k) gd->g[k] = 0.0;
  gd->hinv = beta > 0.0 ? 1.0 / beta : 0.0;
  gd->conv = beta <= tol ? 1 : 0;
  gd->done = gd->conv;
}
__global__ void k_gm_first(double* V, int64_t nv, const double* w, const GmDev* gd) {
  if (gd->done) return;
  const double s = gd->hinv;
  GRID_LOOP(i, nv) V[i] = w[i] * s;
}
__global__ __launch_bounds__(kT) void k_resid_part(const double* b, double* w, int64_t n, double* part) {
  __shared__ double sh[4];
  double v = 0.0;
  GRID_LOOP(i, n) {
    const double r = b[i] - w[i];
    w[i] = r;
    v += r * r;
  }
  v = bsum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}
// y = R^-1 g over the completed steps (one thread)
__global__ void k_gm_solve(GmDev* gd) {
  if (threadIdx.x != 0) return;
  const int j = gd->j, M1 = gd->m + 1;
  for (int i = j - 1; i >= 0; --i) {
    double t = gd->g[i];
    for (int k = i + 1; k < j; ++k) t -= gd->H[(int64_t)k * M1 + i] * gd->y[k];
    gd->y[i] = t / gd->H[(int64_t)i * M1 + i];
  }
}
// x += M^-1 (sum_k y_k V_k)
__global__ void k_gm_update(double* x, const double* V, int64_t nv, int64_t n, const GmDev* gd, int pc,
                            const double* pcd) {
  const int j = gd->j;
  if (pc == GPC_BLOCK2) {
    GRID_LOOP(i, n) {
      double a = 0.0, b = 0.0;
      for (int k = 0; k < j; ++k) {
        a += gd->y[k] * V[(int64_t)k * nv + i];
        b += gd->y[k] * V[(int64_t)k * nv + n + i];
      }
      x[i] += pcd[i] * a + pcd[n + i] * b;
      x[n + i] += pcd[2 * n + i] * a + pcd[3 * n + i] * b;
    }
  } else {
    GRID_LOOP(i, nv) {
      double a = 0.0;
      for (int k = 0; k < j; ++k) a += gd->y[k] * V[(int64_t)k * nv + i];
      x[i] += pc == GPC_JACOBI ? pcd[i] * a : a;
    }
  }
}

// pin = V_j (Schur preconditioner input)
__global__ void k_gm_copyj(const double* V, int64_t nv, double* out, const GmDev* gd) {
  if (gd->done) return;
  const double* v = V + (int64_t)gd->j * nv;
  GRID_LOOP(i, nv) out[i] = v[i];
}
// out = sum_k y_k V_k
__global__ void k_gm_combine(double* out, const double* V, int64_t nv, const GmDev* gd) {
  const int j = gd->j;
  GRID_LOOP(i, nv) {
    double a = 0.0;
    for (int k = 0; k < j; ++k) a += gd->y[k] * V[(int64_t)k * nv + i];
    out[i] = a;
  }
}
// dphi = s t (into the output and into the phi block of pz, whose mu block stays 0)
__global__ void k_sc_phi(double* out, double* pz, const double* t, double s, int64_t n) {
  GRID_LOOP(i, n) {
    const double v = s * t[i];
    out[i] = v;
    pz[i] = v;
  }
}
// Chebyshev iteration for M x = r (Jacobi-scaled, zero start), fixed degree:
// start: r = v_mu - C dphi, x = 0, d = D^-1 r / theta
__global__ void k_ch_start(double* r, double* x, double* d, const double* v_mu, const double* cdphi,
                           const double* dinv, double theta, int64_t n) {
  GRID_LOOP(i, n) {
    const double ri = v_mu[i] - cdphi[i];
    r[i] = ri;
    x[i] = 0.0;
    d[i] = dinv[i] * ri / theta;
  }
}
// x += d; r -= M d (md); d = c1 d + c2 D^-1 r
__global__ void k_ch_step(double* x, double* r, double* d, const double* md, const double* dinv, double c1, double c2,
                          int64_t n) {
  GRID_LOOP(i, n) {
    const double di = d[i];
    x[i] += di;
    const double ri = r[i] - md[i];
    r[i] = ri;
    d[i] = c1 * di + c2 * dinv[i] * ri;
  }
}
// out = s (x + d)  (the last step's x update folded in)
__global__ void k_ch_finish(double* out, const double* x, const double* d, double s, int64_t n) {
  GRID_LOOP(i, n) out[i] = s * (x[i] + d[i]);
}
// lambda_i = (M 1)_i / M_ii (Gershgorin row bound of D^-1 M, all entries >= 0)
__global__ void k_ratio(double* out, const double* ml, const double* dinv, int64_t n) {
  GRID_LOOP(i, n) out[i] = ml[i] * dinv[i];
}

struct Clock {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

int ensure_stepper(Ctx& c, int m) {
  if (!c.step) c.step = new Stepper();
  Stepper& S = *c.step;
  const int64_t n = c.dm.n;
  const int dim = c.dm.dim;
  if (!S.gd) {
    S.n = n;
    S.nv = std::max(2, dim) * n;
    auto A = [&](int64_t cnt) { return (double*)c.dalloc(sizeof(double) * (size_t)std::max<int64_t>(cnt, 1)); };
    S.z = A(S.nv);
    S.w = A(S.nv);
    S.part = A((int64_t)(kGmMax + 1) * kMaxBlocks);
    S.red = A(8);
    S.gd = (GmDev*)c.dalloc(sizeof(GmDev));
    S.X = A(2 * n);
    S.R = A(2 * n);
    S.dX = A(2 * n);
    S.rhs = A(S.nv);
    S.uhat = A(dim * n);
    S.ut = A(dim * n);
    S.unew = A(dim * n);
    S.v = A(dim * n);
    S.pnew = A(n);
    S.phit = A(n);
    S.mut = A(n);
    S.ycoord = A(n);
    S.tmp = A(S.nv);
    S.zero = A(S.nv);
    S.blk = A(4 * n);
    S.binv = A(4 * n);
    S.dvp = A(dim * n);
    S.dvu = A(dim * n);
    S.dm = A(n);
    if (!S.z || !S.w || !S.part || !S.red || !S.gd || !S.X || !S.R || !S.dX || !S.rhs || !S.uhat || !S.ut ||
        !S.unew || !S.v || !S.pnew || !S.phit || !S.mut || !S.ycoord || !S.tmp || !S.zero || !S.blk || !S.binv ||
        !S.dvp || !S.dvu || !S.dm)
      return CHNS_ENOMEM;
    CHNS_HIP(hipHostMalloc((void**)&S.gd_host, sizeof(GmDev), hipHostMallocDefault));
    CHNS_HIP(hipHostMalloc((void**)&S.red_host, sizeof(double) * 8, hipHostMallocDefault));
    for (auto& e : S.ev) CHNS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // vertical coordinate of every node (energy), zeros
    std::vector<double> y((size_t)n);
    const int ax = std::min(std::max(c.prm.gravity_axis, 0), dim - 1);
    const double side = (double)(1 << c.host->max_level);
    for (int64_t i = 0; i < n; ++i) y[(size_t)i] = (double)c.host->indep_coords[3 * i + ax] / side;
    CHNS_HIP(hipMemcpy(S.ycoord, y.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    CHNS_HIP(hipMemset(S.zero, 0, sizeof(double) * S.nv));
  }
  if (m > S.m) {
    S.V = (double*)c.dalloc(sizeof(double) * (size_t)(m + 1) * (size_t)S.nv);
    if (!S.V) return CHNS_ENOMEM;
    S.m = m;
    for (auto& g : S.graphs) (void)hipGraphExecDestroy(g.exec);
    S.graphs.clear();
  }
  return CHNS_OK;
}

// device dot (b == nullptr: sum of a), synchronising
int dot_sync(Ctx& c, const double* a, const double* b, int64_t n, hipStream_t s, double* out) {
  Stepper& S = *c.step;
  const unsigned g = blocks_for(n);
  k_dot_part<<<g, kT, 0, s>>>(a, b, n, S.part);
  k_sum_part<<<1, kT, 0, s>>>(S.part, (int)g, S.red);
  CHNS_HIP(hipGetLastError());
  CHNS_HIP(hipMemcpyAsync(S.red_host, S.red, sizeof(double), hipMemcpyDeviceToHost, s));
  CHNS_HIP(hipStreamSynchronize(s));
  *out = S.red_host[0];
  return CHNS_OK;
}

// Block lower-triangular preconditioner of the Cahn-Hilliard Jacobian
// J = [[A, B], [C, D]] (A = M/dt - advection/2, B = K/(2 Pe Cn),
// C = (M_psi'' + Cn^2 K)/2, D = -M/2):
//   dphi = S~^-1 v_phi,  dmu = D^-1 (v_mu - C dphi),  D^-1 = -2 M^-1,
// with the Schur complement S = A - B D^-1 C approximated, dropping the
// advection and psi'' parts, by (1/dt)(M + sqrt(b) K) M^-1 (M + sqrt(b) K),
// b = dt Cn / (2 Pe):  S~^-1 = (dt/b) A_g^-1 M A_g^-1, A_g = K + M/sqrt(b),
// each A_g^-1 one multigrid V-cycle of the pressure hierarchy set up with
// rho = 1 and the mass shift 1/sqrt(b).  C dphi is the mu block of J [dphi, 0].
// A fixed linear map (fixed cycles), so plain right-preconditioned GMRES
// applies.  in / out: 2n, in = [v_phi, v_mu].
constexpr int kMassCheb = 12;  // Chebyshev degree of the mass solve
int ch_schur_apply(Ctx& c, const double* in, double* out, hipStream_t s) {
  Stepper& S = *c.step;
  const int64_t n = c.dm.n;
  const unsigned g = blocks_ew(n);
  int rc;
  ApplyOut plain{};
  if ((rc = mg_vcycle64(c, in, S.pt1, s))) return rc;
  if ((rc = launch_apply(c, CHNS_OP_MASS, CHNS_FP64, S.pt1, S.pt2, s, plain))) return rc;
  if ((rc = mg_vcycle64(c, S.pt2, S.pt1, s))) return rc;
  k_sc_phi<<<g, kT, 0, s>>>(out, S.pz, S.pt1, S.sc_scale, n);
  CHNS_HIP(hipGetLastError());
  if ((rc = launch_apply(c, CHNS_OP_CH_JACOBIAN, CHNS_FP64, S.pz, S.pj, s, plain))) return rc;
  // dmu = -2 M^-1 (v_mu - C dphi): Chebyshev on [lmax / 27, lmax] (the
  // Jacobi-scaled Q1 mass spectrum spans a factor 3^d on uniform meshes)
  const double lmax = S.m_lmax, lmin = lmax / (c.dm.dim == 3 ? 27.0 : 9.0);
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  k_ch_start<<<g, kT, 0, s>>>(S.cr, S.cx, S.cd, in + n, S.pj + n, S.dMinv, theta, n);
  double rho = 1.0 / sigma;
  for (int k = 1; k < kMassCheb; ++k) {
    if ((rc = launch_apply(c, CHNS_OP_MASS, CHNS_FP64, S.cd, S.pt2, s, plain))) return rc;
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    k_ch_step<<<g, kT, 0, s>>>(S.cx, S.cr, S.cd, S.pt2, S.dMinv, rho1 * rho, 2.0 * rho1 / delta, n);
    rho = rho1;
  }
  k_ch_finish<<<g, kT, 0, s>>>(out + n, S.cx, S.cd, -2.0, n);
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

// input/output vectors of the multigrid-based GMRES preconditioners (up to
// three fields)
int ensure_pc_io(Ctx& c) {
  Stepper& S = *c.step;
  const size_t bytes = sizeof(double) * 3 * (size_t)c.dm.n;
  if (!S.pin) S.pin = (double*)c.dalloc(bytes);
  if (!S.pout) S.pout = (double*)c.dalloc(bytes);
  return S.pin && S.pout ? CHNS_OK : CHNS_ENOMEM;
}

__global__ void k_mask_walls(const double* __restrict__ in, const uint8_t* __restrict__ wall, double* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    out[i] = wall[i] ? 0.0 : in[i];
}
__global__ void k_wall_rows(double* z, const double* __restrict__ in, const uint8_t* __restrict__ wall, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    if (wall[i]) z[i] = in[i];
}

// Momentum preconditioner: per velocity component, one V-cycle of the
// scalar operator rho/dt M + eta/(2 Re) K (natural boundary rows, set up by
// vp_mg_setup) on the input with its wall entries dropped; the wall rows of
// the momentum operator are the identity, so they pass the input through.
int vp_mg_apply(Ctx& c, const double* in, double* out, hipStream_t s) {
  Stepper& S = *c.step;
  const int64_t n = c.dm.n;
  const unsigned g = blocks_for(n);
  for (int d = 0; d < c.dm.dim; ++d) {
    k_mask_walls<<<g, kT, 0, s>>>(in + d * n, c.dm.wall, S.vmask, n);
    CHNS_HIP(hipGetLastError());
    int rc = mg_vcycle64(c, S.vmask, out + d * n, s);
    if (rc) return rc;
    k_wall_rows<<<g, kT, 0, s>>>(out + d * n, in + d * n, c.dm.wall, n);
    CHNS_HIP(hipGetLastError());
  }
  return CHNS_OK;
}

// Multigrid hierarchy of the scalar momentum operator at the context's
// phase field; the caller restores the pressure operator afterwards.
int vp_mg_setup(Ctx& c, hipStream_t s) {
  Stepper& S = *c.step;
  int rc;
  if ((rc = ensure_pc_io(c))) return rc;
  if (!S.vmask && !(S.vmask = (double*)c.dalloc(sizeof(double) * (size_t)c.dm.n))) return CHNS_ENOMEM;
  if ((rc = mg_build(c))) return rc;
  c.pp_kind = 1;
  c.pp_shift = 0.0;
  c.mg->setup_valid = false;
  return mg_setup(c, s);
}

// Restarted right-preconditioned GMRES(m) on A x = b, A = the public
// operator `op` with its current coefficient fields; x in/out.
int gmres(Ctx& c, int op, const double* b, double* x, int pc, const double* pcd, double rtol, int max_it, int m,
          bool graphs, hipStream_t s, int* iters, double* rel) {
  Stepper& S = *c.step;
  const int64_t n = c.dm.n;
  const int64_t nv = n * op_fields(op, c.dm.dim);
  const unsigned g = blocks_for(nv);
  const unsigned gn = blocks_for(n);
  int rc;
  double bb = 0.0;
  if ((rc = dot_sync(c, b, b, nv, s, &bb))) return rc;
  *iters = 0;
  *rel = 0.0;
  if (bb == 0.0) {
    k_fill0<<<g, kT, 0, s>>>(x, nv);
    CHNS_HIP(hipGetLastError());
    return CHNS_OK;
  }
  const double bn = std::sqrt(bb);
  const double tol = rtol * bn;
  ApplyOut plain{};
  ApplyOut gated{};
  gated.done = &S.gd->done;
  auto step = [&](hipStream_t st) -> int {
    int e;
    if (pc == GPC_SCHUR || pc == GPC_VPMG) {
      k_gm_copyj<<<blocks_ew(nv), kT, 0, st>>>(S.V, nv, S.pin, S.gd);
      CHNS_HIP(hipGetLastError());
      if ((e = pc == GPC_SCHUR ? ch_schur_apply(c, S.pin, S.z, st) : vp_mg_apply(c, S.pin, S.z, st))) return e;
    } else {
      k_gm_pc<<<blocks_ew(pc == GPC_BLOCK2 ? n : nv), kT, 0, st>>>(S.V, nv, n, S.z, S.gd, pc, pcd);
      CHNS_HIP(hipGetLastError());
    }
    e = launch_apply(c, op, CHNS_FP64, S.z, S.w, st, gated);
    if (e) return e;
    for (int pass = 1; pass <= 2; ++pass) {
      k_gm_multidot<<<g, kT, 0, st>>>(S.V, nv, S.w, S.gd, S.part);
      k_gm_fin<<<kGmMax + 1, kT, 0, st>>>(S.part, (int)g, S.gd, pass);
      k_gm_orth<<<g, kT, 0, st>>>(S.V, nv, S.w, S.gd, pass, S.part);
      CHNS_HIP(hipGetLastError());
    }
    k_gm_givens<<<1, kT, 0, st>>>(S.part, (int)g, S.gd);
    k_gm_scale<<<blocks_ew(nv), kT, 0, st>>>(S.V, nv, S.w, S.gd);
    CHNS_HIP(hipGetLastError());
    return CHNS_OK;
  };
  hipGraphExec_t exec = nullptr;
  if (graphs && !c.prof) {
    for (auto& ge : S.graphs)
      if (ge.op == op && ge.pc == pc && ge.pcdata == (const void*)pcd) exec = ge.exec;
    if (!exec) {
      hipGraph_t gr = nullptr;
      CHNS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
      int e = step(s);
      hipError_t ce = hipStreamEndCapture(s, &gr);
      if (e) return e;
      if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
      hipError_t ie = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
      S.graphs.push_back({op, pc, (const void*)pcd, exec});
    }
  }
  const int depth = 4;
  int total = 0;
  while (true) {
    // true residual, first basis vector
    if ((rc = launch_apply(c, op, CHNS_FP64, x, S.w, s, plain))) return rc;
    k_resid_part<<<g, kT, 0, s>>>(b, S.w, nv, S.part);
    k_gm_start<<<1, kT, 0, s>>>(S.part, (int)g, S.gd, tol, m);
    k_gm_first<<<g, kT, 0, s>>>(S.V, nv, S.w, S.gd);
    CHNS_HIP(hipGetLastError());
    CHNS_HIP(hipMemcpyAsync(S.gd_host, S.gd, 64, hipMemcpyDeviceToHost, s));
    CHNS_HIP(hipStreamSynchronize(s));
    *rel = S.gd_host->beta / bn;
    if (!std::isfinite(*rel)) {
      set_error("GMRES: the residual is not finite");
      return CHNS_ENOCONV;
    }
    if (S.gd_host->conv || total >= max_it) break;
    // Arnoldi steps until the device flags the end of the cycle
    for (int it = 0; it < m; ++it) {
      if (exec) {
        CHNS_HIP(hipGraphLaunch(exec, s));
      } else if ((rc = step(s))) {
        return rc;
      }
      CHNS_HIP(hipMemcpyAsync(&S.gd_host[0], S.gd, 16, hipMemcpyDeviceToHost, s));
      if (it % depth == depth - 1 || it == m - 1) {
        CHNS_HIP(hipStreamSynchronize(s));
        if (S.gd_host->done) break;
      }
    }
    CHNS_HIP(hipStreamSynchronize(s));
    total += S.gd_host->j;
    k_gm_solve<<<1, 64, 0, s>>>(S.gd);
    if (pc == GPC_SCHUR || pc == GPC_VPMG) {
      k_gm_combine<<<g, kT, 0, s>>>(S.pin, S.V, nv, S.gd);
      CHNS_HIP(hipGetLastError());
      if ((rc = pc == GPC_SCHUR ? ch_schur_apply(c, S.pin, S.pout, s) : vp_mg_apply(c, S.pin, S.pout, s))) return rc;
      k_add<<<g, kT, 0, s>>>(x, S.pout, nv);
    } else {
      k_gm_update<<<pc == GPC_BLOCK2 ? gn : g, kT, 0, s>>>(x, S.V, nv, n, S.gd, pc, pcd);
    }
    CHNS_HIP(hipGetLastError());
  }
  *iters = total;
  if (!(*rel <= rtol)) {
    set_error("GMRES did not reach rtol");
    return CHNS_ENOCONV;
  }
  return CHNS_OK;
}

int copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  CHNS_HIP(hipMemcpyAsync(dst, src, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
  return CHNS_OK;
}

int ensure_coef(Ctx& c, double** buf) {
  if (!*buf) *buf = (double*)c.dalloc(sizeof(double) * (size_t)(2 + c.dm.dim) * (size_t)c.dm.n);
  return *buf ? CHNS_OK : CHNS_ENOMEM;
}

// Newton iteration for the Cahn-Hilliard block: X = [phi, mu] holds the
// guess on entry and the iterate on exit (Def. 6; x <- x - J^-1 R until
// |R| <= max(rtol |R_0|, atol)).
// Multigrid hierarchy for the Schur preconditioner: rho = 1 (phase field 1)
// and the mass shift 1/sqrt(b); lumped mass and work vectors on first use.
// The pressure solve of the step sets its own phase field afterwards, which
// invalidates this set-up.
int schur_setup(Ctx& c, hipStream_t s) {
  Stepper& S = *c.step;
  const int64_t n = c.dm.n;
  int rc;
  if (!S.mL) {
    auto A = [&](int64_t cnt) { return (double*)c.dalloc(sizeof(double) * (size_t)cnt); };
    S.mL = A(n);
    S.dMinv = A(n);
    S.cx = A(n);
    S.cr = A(n);
    S.cd = A(n);
    if (!S.dMinv || !S.cx || !S.cr || !S.cd) return CHNS_ENOMEM;
    if ((rc = ensure_pc_io(c))) return rc;
    S.pt1 = A(n);
    S.pt2 = A(n);
    S.pz = A(2 * n);
    S.pj = A(2 * n);
    if (!S.mL || !S.pt1 || !S.pt2 || !S.pz || !S.pj) return CHNS_ENOMEM;
    // the mu block of pz stays zero; lumped mass M 1
    k_fill0<<<blocks_for(2 * n), kT, 0, s>>>(S.pz, 2 * n);
    k_fill1<<<blocks_for(n), kT, 0, s>>>(S.pt2, n);
    CHNS_HIP(hipGetLastError());
    ApplyOut plain{};
    if ((rc = launch_apply(c, CHNS_OP_MASS, CHNS_FP64, S.pt2, S.mL, s, plain))) return rc;
    // inverse mass diagonal and the Gershgorin bound max_i (M 1)_i / M_ii
    if ((rc = launch_diagonal(c, CHNS_OP_MASS, CHNS_FP64, S.dMinv, true, s))) return rc;
    k_ratio<<<blocks_for(n), kT, 0, s>>>(S.pt1, S.mL, S.dMinv, n);
    CHNS_HIP(hipGetLastError());
    std::vector<double> ratio((size_t)n);
    CHNS_HIP(hipMemcpyAsync(ratio.data(), S.pt1, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    CHNS_HIP(hipStreamSynchronize(s));
    S.m_lmax = *std::max_element(ratio.begin(), ratio.end());
  }
  const double Pe = c.prm.Pe > 0.0 ? c.prm.Pe : 1.0 / (3.0 * c.prm.Cn * c.prm.Cn);
  const double b = c.prm.dt * c.prm.Cn / (2.0 * Pe);
  S.sc_scale = c.prm.dt / b;
  if ((rc = mg_build(c))) return rc;
  k_fill1<<<blocks_for(n), kT, 0, s>>>(S.pt1, n);
  CHNS_HIP(hipGetLastError());
  if ((rc = launch_set_phase(c, S.pt1, nullptr, s))) return rc;
  c.pp_shift = 1.0 / std::sqrt(b);
  rc = mg_setup(c, s);
  return rc;
}

int newton_ch_impl(Ctx& c, const double* phi0, const double* mu0, const double* ut, const double* fch,
                   const chns_step_opts& o, bool graphs, hipStream_t s, int* newton_it, int* lin_it, double* rfinal);

// the mass shift is the pressure operator's only while the Newton solve runs
int newton_ch(Ctx& c, const double* phi0, const double* mu0, const double* ut, const double* fch,
              const chns_step_opts& o, bool graphs, hipStream_t s, int* newton_it, int* lin_it, double* rfinal) {
  const int rc = newton_ch_impl(c, phi0, mu0, ut, fch, o, graphs, s, newton_it, lin_it, rfinal);
  if (c.pp_shift != 0.0) {
    c.pp_shift = 0.0;
    c.diag_valid = false;
    if (c.mg) c.mg->setup_valid = false;
  }
  return rc;
}

// fch (nullable): body-force vector added to every residual (2n)
int newton_ch_impl(Ctx& c, const double* phi0, const double* mu0, const double* ut, const double* fch,
                   const chns_step_opts& o, bool graphs, hipStream_t s, int* newton_it, int* lin_it, double* rfinal) {
  Stepper& S = *c.step;
  const int64_t n = c.dm.n;
  const int dim = c.dm.dim;
  const unsigned g2 = blocks_for(2 * n);
  const double* cf[kMaxCoefFields] = {};
  cf[0] = phi0;
  cf[1] = mu0;
  for (int d = 0; d < dim; ++d) cf[2 + d] = ut + d * n;
  ApplyOut plain{};
  int rc;
  double rr = 0.0;
  if ((rc = launch_form(c, FORM_CH_RES, S.X, cf, S.R, s, plain))) return rc;
  if (fch) k_add<<<g2, kT, 0, s>>>(S.R, fch, 2 * n);
  if ((rc = dot_sync(c, S.R, S.R, 2 * n, s, &rr))) return rc;
  const double r0 = std::sqrt(rr);
  double rn = r0;
  int it = 0;
  *newton_it = 0;
  *rfinal = rn;
  if (!std::isfinite(r0)) {
    set_error("Cahn-Hilliard residual is not finite (NaN or infinity in the state)");
    return CHNS_ENOCONV;
  }
  if ((rc = ensure_coef(c, &c.coef_chj))) return rc;
  const bool schur = o.ch_pc == CHNS_CH_PC_SCHUR_GMG;
  if (schur && (rc = schur_setup(c, s))) return rc;
  const double ntol = std::max(o.newton_rtol * r0, o.newton_atol);
  while (!(rn <= ntol) && it < o.max_newton) {
    // Jacobian coefficients [phi~ = (phi^{k+1} + phi^k)/2, u~] and its 2x2
    // node blocks
    k_axpby<<<blocks_for(n), kT, 0, s>>>(c.coef_chj, 0.5, S.X, 0.5, phi0, n);
    CHNS_HIP(hipGetLastError());
    if ((rc = copy(c.coef_chj + n, ut, dim * n, s))) return rc;
    c.coef_chj_set = true;
    c.coef_chj32_ok = false;
    for (int k = 6; k < 8; ++k) {
      if (!c.w64[k]) c.w64[k] = (double*)c.dalloc(sizeof(double) * n * 3);
      if (!c.w64[k]) return CHNS_ENOMEM;
    }
    if (!schur) {
      if ((rc = launch_block_diagonal(c, CHNS_OP_CH_JACOBIAN, S.blk, c.w64[6], c.w64[7], s))) return rc;
      k_inv2<<<blocks_for(n), kT, 0, s>>>(S.blk, S.binv, n);
    }
    k_scal<<<g2, kT, 0, s>>>(S.rhs, -1.0, S.R, 2 * n);
    k_fill0<<<g2, kT, 0, s>>>(S.dX, 2 * n);
    CHNS_HIP(hipGetLastError());
    int li = 0;
    double rel = 0.0;
    rc = gmres(c, CHNS_OP_CH_JACOBIAN, S.rhs, S.dX, schur ? GPC_SCHUR : GPC_BLOCK2, schur ? S.mL : S.binv,
               o.lin_rtol, o.max_it, o.restart, graphs, s, &li, &rel);
    *lin_it += li;
    if (rc) return rc;
    k_add<<<g2, kT, 0, s>>>(S.X, S.dX, 2 * n);
    CHNS_HIP(hipGetLastError());
    if ((rc = launch_form(c, FORM_CH_RES, S.X, cf, S.R, s, plain))) return rc;
  if (fch) k_add<<<g2, kT, 0, s>>>(S.R, fch, 2 * n);
    if ((rc = dot_sync(c, S.R, S.R, 2 * n, s, &rr))) return rc;
    rn = std::sqrt(rr);
    ++it;
  }
  *newton_it = it;
  *rfinal = rn;
  if (!(rn <= ntol)) {
    set_error("Newton iteration for the Cahn-Hilliard system did not converge");
    return CHNS_ENOCONV;
  }
  return CHNS_OK;
}

}  // namespace

void destroy_stepper(Ctx& c) {
  if (!c.step) return;
  Stepper& S = *c.step;
  for (auto& g : S.graphs) (void)hipGraphExecDestroy(g.exec);
  for (auto e : S.ev)
    if (e) (void)hipEventDestroy(e);
  if (S.gd_host) (void)hipHostFree(S.gd_host);
  if (S.red_host) (void)hipHostFree(S.red_host);
  delete c.step;
  c.step = nullptr;
}

int set_coefficients_impl(Ctx& c, int op, const double* const* fields, hipStream_t s) {
  const int64_t n = c.dm.n;
  const int dim = c.dm.dim;
  if (op != CHNS_OP_MOMENTUM && op != CHNS_OP_CH_JACOBIAN) {
    set_error("coefficients are set for CHNS_OP_MOMENTUM and CHNS_OP_CH_JACOBIAN only");
    return CHNS_EINVAL;
  }
  if (!fields || !fields[0] || !fields[1] || !fields[2]) {
    set_error("null coefficient field");
    return CHNS_EINVAL;
  }
  double** buf = op == CHNS_OP_MOMENTUM ? &c.coef_mom : &c.coef_chj;
  int rc;
  if ((rc = ensure_coef(c, buf))) return rc;
  if (op == CHNS_OP_MOMENTUM) {
    if ((rc = copy(*buf, fields[0], n, s))) return rc;
    if ((rc = copy(*buf + n, fields[1], n, s))) return rc;
    if ((rc = copy(*buf + 2 * n, fields[2], dim * n, s))) return rc;
  } else {
    // the Jacobian reads phi^{k+1} and phi^k only through their average
    k_axpby<<<blocks_for(n), kT, 0, s>>>(*buf, 0.5, fields[0], 0.5, fields[1], n);
    CHNS_HIP(hipGetLastError());
    if ((rc = copy(*buf + n, fields[2], dim * n, s))) return rc;
  }
  (op == CHNS_OP_MOMENTUM ? c.coef_mom_set : c.coef_chj_set) = true;
  (op == CHNS_OP_MOMENTUM ? c.coef_mom32_ok : c.coef_chj32_ok) = false;
  return CHNS_OK;
}

int assemble_impl(Ctx& c, int form, const double* const* fields, double* out, hipStream_t s) {
  const int64_t n = c.dm.n;
  const int dim = c.dm.dim;
  int rc;
  if ((rc = ensure_stepper(c, 1))) return rc;
  const double* cf[kMaxCoefFields] = {};
  int need = 0;
  switch (form) {
    case CHNS_FORM_CH_RESIDUAL: need = 4; break;
    case CHNS_FORM_VP_RHS: need = 5; break;
    case CHNS_FORM_PP_RHS: need = 6; break;
    case CHNS_FORM_VU_RHS: need = 7; break;
    case CHNS_FORM_ENERGY: need = 2; break;
    default:
      set_error("unknown form");
      return CHNS_EINVAL;
  }
  if (!fields || !out) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  for (int k = 0; k < need; ++k)
    if (!fields[k]) {
      set_error("null field");
      return CHNS_EINVAL;
    }
  ApplyOut plain{};
  if (form == CHNS_FORM_CH_RESIDUAL) {
    cf[0] = fields[1];
    cf[1] = fields[2];
    for (int d = 0; d < dim; ++d) cf[2 + d] = fields[3] + d * n;
    return launch_form(c, FORM_CH_RES, fields[0], cf, out, s, plain);
  }
  if (form == CHNS_FORM_ENERGY) {
    cf[0] = fields[0];
    cf[1] = c.step->ycoord;
    for (int d = 0; d < dim; ++d) cf[2 + d] = fields[1] + d * n;
    return launch_form(c, FORM_ENERGY, nullptr, cf, out, s, plain);
  }
  // phi~, mu~, u^ (dim), u^k (dim), p^k, v (dim), p^{k+1}
  int k = 0;
  cf[k++] = fields[0];
  cf[k++] = fields[1];
  for (int d = 0; d < dim; ++d) cf[k++] = fields[2] + d * n;
  for (int d = 0; d < dim; ++d) cf[k++] = fields[3] + d * n;
  cf[k++] = fields[4];
  if (form >= CHNS_FORM_PP_RHS)
    for (int d = 0; d < dim; ++d) cf[k++] = fields[5] + d * n;
  if (form == CHNS_FORM_VU_RHS) cf[k++] = fields[6];
  for (int d = 0; d < dim; ++d) cf[k++] = c.step->zero;  // no body force
  const int f = form == CHNS_FORM_VP_RHS ? FORM_VP_RHS : (form == CHNS_FORM_PP_RHS ? FORM_PP_RHS : FORM_VU_RHS);
  return launch_form(c, f, nullptr, cf, out, s, plain);
}

int initial_mu_impl(Ctx& c, const double* phi, double* mu, hipStream_t s) {
  const int64_t n = c.dm.n;
  const int dim = c.dm.dim;
  int rc;
  if ((rc = ensure_stepper(c, 1))) return rc;
  Stepper& S = *c.step;
  // mu-block of the CH residual at phi^{k+1} = phi^k = phi, mu = 0, u = 0:
  // (q, psi'(phi)) + Cn^2 (grad q, grad phi)
  const double* cf[kMaxCoefFields] = {};
  cf[0] = phi;
  cf[1] = S.zero;
  for (int d = 0; d < dim; ++d) cf[2 + d] = S.zero;
  if ((rc = copy(S.X, phi, n, s))) return rc;
  k_fill0<<<blocks_for(n), kT, 0, s>>>(S.X + n, n);
  CHNS_HIP(hipGetLastError());
  ApplyOut plain{};
  if ((rc = launch_form(c, FORM_CH_RES, S.X, cf, S.R, s, plain))) return rc;
  // M mu = rhs by Jacobi-CG on the plain mass matrix
  if ((rc = launch_diagonal(c, CHNS_OP_MASS, CHNS_FP64, S.dm, true, s))) return rc;
  k_fill0<<<blocks_for(n), kT, 0, s>>>(mu, n);
  CHNS_HIP(hipGetLastError());
  int it = 0;
  double rel = 0.0;
  return solve_spd_impl(c, CHNS_OP_MASS, S.R + n, mu, S.dm, 1e-13, 10000, false, s, &it, &rel);
}

int advance_step_body(Ctx& c, const chns_state& st, const chns_step_opts& o, chns_step_stats& stats,
                      hipStream_t caller);

// On an error return the step has replaced the context's phase field (and
// possibly the operator behind the multigrid hierarchy) part way through:
// the phase field is marked unset, so later pressure applies and solves
// return CHNS_ESTATE until chns_set_phase_field, and every cached set-up is
// invalidated.
int advance_step_impl(Ctx& c, const chns_state& st, const chns_step_opts& o, chns_step_stats& stats,
                      hipStream_t caller) {
  const int rc = advance_step_body(c, st, o, stats, caller);
  if (rc) {
    c.phi_set = false;
    c.pp_kind = 0;
    c.pp_shift = 0.0;
    c.diag_valid = false;
    if (c.mg) c.mg->setup_valid = false;
  }
  return rc;
}

int advance_step_body(Ctx& c, const chns_state& st, const chns_step_opts& o, chns_step_stats& stats,
                      hipStream_t caller) {
  Clock clk;
  const int64_t n = c.dm.n;
  const int dim = c.dm.dim;
  int rc;
  if (o.restart < 1 || o.restart > kGmMax) {
    set_error("GMRES restart length must be in [1, 128]");
    return CHNS_EINVAL;
  }
  if ((rc = ensure_stepper(c, o.restart))) return rc;
  Stepper& S = *c.step;
  CHNS_HIP(hipEventRecord(c.ev_in, caller));
  CHNS_HIP(hipStreamWaitEvent(c.work, c.ev_in, 0));
  hipStream_t s = c.work;
  const bool graphs = o.no_graphs == 0;
  const unsigned gv = blocks_for(dim * n);
  const unsigned g1 = blocks_for(n);
  ApplyOut plain{};
  // u^ = (3 u^k - u^{k-1}) / 2, u^{k+1} := u^k, X = [phi^k, mu^k], p^{k+1} := p^k
  k_axpby<<<gv, kT, 0, s>>>(S.uhat, 1.5, st.u, -0.5, st.u_prev, dim * n);
  CHNS_HIP(hipGetLastError());
  if ((rc = copy(S.unew, st.u, dim * n, s))) return rc;
  if ((rc = copy(S.X, st.phi, n, s))) return rc;
  if ((rc = copy(S.X + n, st.mu, n, s))) return rc;
  if ((rc = copy(S.pnew, st.p, n, s))) return rc;
  stats = chns_step_stats{};
  // body forces of the Cahn-Hilliard system: R_phi -= M f_phi, R_mu += M f_mu
  const double* fch = nullptr;
  if (o.force_phi || o.force_mu) {
    if (!S.fch && !(S.fch = (double*)c.dalloc(sizeof(double) * 2 * (size_t)n))) return CHNS_ENOMEM;
    k_fill0<<<blocks_for(2 * n), kT, 0, s>>>(S.fch, 2 * n);
    CHNS_HIP(hipGetLastError());
    if (o.force_phi) {
      if ((rc = launch_apply(c, CHNS_OP_MASS, CHNS_FP64, o.force_phi, S.tmp, s, plain))) return rc;
      k_axpby<<<g1, kT, 0, s>>>(S.fch, -1.0, S.tmp, 0.0, S.tmp, n);
    }
    if (o.force_mu && (rc = launch_apply(c, CHNS_OP_MASS, CHNS_FP64, o.force_mu, S.fch + n, s, plain))) return rc;
    CHNS_HIP(hipGetLastError());
    fch = S.fch;
  }
  for (int blk = 0; blk < o.blocks; ++blk) {
    // ---- Cahn-Hilliard with u~ = (u^k + u^{k+1}) / 2
    k_axpby<<<gv, kT, 0, s>>>(S.ut, 0.5, st.u, 0.5, S.unew, dim * n);
    CHNS_HIP(hipGetLastError());
    int nit = 0;
    double rfin = 0.0;
    rc = newton_ch(c, st.phi, st.mu, S.ut, fch, o, graphs, s, &nit, &stats.ch_iterations, &rfin);
    if (blk < 4) stats.newton_iterations[blk] = nit;
    stats.ch_residual = rfin;
    if (rc) return rc;
    // ---- time-averaged phase field and chemical potential
    k_axpby<<<g1, kT, 0, s>>>(S.phit, 0.5, S.X, 0.5, st.phi, n);
    k_axpby<<<g1, kT, 0, s>>>(S.mut, 0.5, S.X + n, 0.5, st.mu, n);
    CHNS_HIP(hipGetLastError());
    // ---- velocity prediction
    const double* cf[kMaxCoefFields] = {};
    int k = 0;
    cf[k++] = S.phit;
    cf[k++] = S.mut;
    for (int d = 0; d < dim; ++d) cf[k++] = S.uhat + d * n;
    for (int d = 0; d < dim; ++d) cf[k++] = st.u + d * n;
    cf[k++] = st.p;
    // body force of the momentum equation after each form's own fields
    auto force_at = [&](int k0) {
      for (int d = 0; d < dim; ++d) cf[k0 + d] = o.force_v ? o.force_v + d * n : S.zero;
    };
    force_at(k);
    if ((rc = launch_form(c, FORM_VP_RHS, nullptr, cf, S.rhs, s, plain))) return rc;
    if ((rc = ensure_coef(c, &c.coef_mom))) return rc;
    if ((rc = copy(c.coef_mom, S.phit, n, s))) return rc;
    if ((rc = copy(c.coef_mom + n, S.mut, n, s))) return rc;
    if ((rc = copy(c.coef_mom + 2 * n, S.uhat, dim * n, s))) return rc;
    c.coef_mom_set = true;
    c.coef_mom32_ok = false;
    // phase field phi~ of the pressure solve (and of the momentum multigrid)
    if ((rc = launch_set_phase(c, S.X, st.phi, s))) return rc;
    const bool vpmg = o.vp_pc == CHNS_VP_PC_GMG;
    if (vpmg) {
      rc = vp_mg_setup(c, s);
    } else {
      rc = launch_diagonal(c, CHNS_OP_MOMENTUM, CHNS_FP64, S.dvp, true, s);
    }
    if (!rc) rc = copy(S.v, st.u, dim * n, s);
    int li = 0;
    double rel = 0.0;
    if (!rc)
      rc = gmres(c, CHNS_OP_MOMENTUM, S.rhs, S.v, vpmg ? GPC_VPMG : GPC_JACOBI, vpmg ? nullptr : S.dvp, o.lin_rtol,
                 o.max_it, o.restart, graphs, s, &li, &rel);
    if (vpmg) {
      // the hierarchy and the operator behind CHNS_OP_PRESSURE return to
      // the pressure Poisson problem
      c.pp_kind = 0;
      c.diag_valid = false;
      if (c.mg) c.mg->setup_valid = false;
    }
    stats.vp_iterations += li;
    if (rc) return rc;
    // ---- pressure Poisson with 1/rho(phi~)
    for (int d = 0; d < dim; ++d) cf[k++] = S.v + d * n;
    force_at(k);
    if ((rc = launch_form(c, FORM_PP_RHS, nullptr, cf, S.rhs, s, plain))) return rc;
    chns_solve_opts po{};
    po.rtol = o.lin_rtol;
    po.max_it = o.max_it;
    po.pc = o.pp_pc;
    po.mode = o.pp_mode;
    po.inner_rtol = 1e-4;
    po.check_every = 16;
    po.max_outer = 30;
    po.no_graphs = o.no_graphs;
    chns_solve_stats ps{};
    rc = solve_pressure_impl(c, S.rhs, S.pnew, po, ps, s);
    stats.pp_iterations += ps.iterations;
    if (rc) return rc;
    // ---- velocity update: M_rho u^{k+1} = ...
    cf[k++] = S.pnew;
    force_at(k);
    if ((rc = launch_form(c, FORM_VU_RHS, nullptr, cf, S.rhs, s, plain))) return rc;
    if ((rc = launch_diagonal(c, CHNS_OP_MASS_RHO, CHNS_FP64, S.dvu, true, s))) return rc;
    if ((rc = copy(S.unew, S.v, dim * n, s))) return rc;
    rc = solve_spd_impl(c, CHNS_OP_MASS_RHO, S.rhs, S.unew, S.dvu, o.lin_rtol, o.max_it, graphs, s, &li, &rel);
    stats.vu_iterations += li;
    if (rc) return rc;
  }
  // new state
  if ((rc = copy(st.u_prev, st.u, dim * n, s))) return rc;
  if ((rc = copy(st.u, S.unew, dim * n, s))) return rc;
  if ((rc = copy(st.p, S.pnew, n, s))) return rc;
  if ((rc = copy(st.phi, S.X, n, s))) return rc;
  if ((rc = copy(st.mu, S.X + n, n, s))) return rc;
  // mass = 1^T M phi, energy = sum of the nodal shares
  if ((rc = launch_apply(c, CHNS_OP_MASS, CHNS_FP64, st.phi, S.tmp, s, plain))) return rc;
  if ((rc = dot_sync(c, S.tmp, nullptr, n, s, &stats.mass))) return rc;
  const double* ef[kMaxCoefFields] = {};
  ef[0] = st.phi;
  ef[1] = S.ycoord;
  for (int d = 0; d < dim; ++d) ef[2 + d] = st.u + d * n;
  if ((rc = launch_form(c, FORM_ENERGY, nullptr, ef, S.tmp, s, plain))) return rc;
  if ((rc = dot_sync(c, S.tmp, nullptr, n, s, &stats.energy))) return rc;
  CHNS_HIP(hipStreamSynchronize(s));
  stats.ms = clk.ms();
  return CHNS_OK;
}

}  // namespace chns
