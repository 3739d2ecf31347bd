// Device-resident Krylov solvers for the pressure Poisson system.
//
// All scalars (dot products, step lengths, iteration count, convergence flag)
// live in device memory; the host only enqueues kernels and polls the flag
// every few iterations.  Dot products are accumulated in FP64 with a
// wavefront + block tree and a last-block finalisation over the per-block
// partials in a fixed order, so every reduction is deterministic.
//
// Solvers:
//   * Jacobi-preconditioned CG (FP64, or FP32 vectors with FP64 dots);
//   * FP64 iterative refinement around FP32 inner CG solves (mixed mode);
// the paper solves the pressure Poisson system with PETSc Krylov methods
// (appendix on solver options); CG is the natural choice for the symmetric
// positive semi-definite operator.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "chns_internal.h"

namespace chns {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-block partial sums of NV doubles: partials[k * kStride + block].  The
// totals are formed by a one-block finalisation kernel launched next on the
// same stream (kernel boundaries order the writes; no per-block fences).
constexpr int kStride = kMaxPartials / 4;
template <int NV>
__device__ void block_partials(double (&v)[NV], double* partials) {
  __shared__ double sh[NV][4];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = wsum(v[k]);
    if ((threadIdx.x & 63) == 0) sh[k][w] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) partials[k * kStride + blockIdx.x] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
  }
}

enum FinMode { FIN_STORE = 0, FIN_CG_INIT = 1, FIN_CG_UPDATE = 2, FIN_FCG_UPDATE = 3, FIN_FCG_CONT = 4 };

// Fixed-order totals of nv partial arrays, then the scalar update of `mode`.
// 1024 threads, each with four independent running sums, so the few thousand
// partials are read with many loads in flight.
constexpr int kFinThreads = 1024;
__global__ __launch_bounds__(kFinThreads) void k_finalize(const double* partials, int nparts, int nv, int mode,
                                                          DevScalars* sc, double* out, int respect_done,
                                                          int* flag_host) {
  __shared__ double sh[kFinThreads / 64];
  if (respect_done && sc->done) return;
  double tot[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < nv; ++k) {
    const double* pk = partials + k * kStride;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * kFinThreads < nparts; b += 4 * kFinThreads) {
      v0 += pk[b];
      v1 += pk[b + kFinThreads];
      v2 += pk[b + 2 * kFinThreads];
      v3 += pk[b + 3 * kFinThreads];
    }
    for (; b < nparts; b += kFinThreads) v0 += pk[b];
    double v = (v0 + v1) + (v2 + v3);
    v = wsum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kFinThreads / 64; ++i) t += sh[i];
    tot[k] = t;
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (mode == FIN_STORE) {
    *out = tot[0];
  } else if (mode == FIN_CG_INIT || mode == FIN_FCG_CONT) {
    sc->rz = tot[0];
    sc->rr = tot[1];
    sc->it = 0;
    // flexible CG continued across a residual replacement: z.r_old for the
    // continued direction (see k_cont_p_flex)
    if (mode == FIN_FCG_CONT) sc->beta = tot[2];
    // converged, or breakdown: a non-finite residual or r.z <= 0 (an
    // indefinite or vanishing preconditioner output) ends the solve at x_0
    sc->done = (tot[1] <= sc->tol2 || !(tot[1] == tot[1]) || !(tot[0] > 0.0)) ? 1 : 0;
  } else {
    // CG: beta = (r_new.z_new) / (r_old.z_old); flexible CG (Polak-Ribiere
    // form): beta = z_new.(r_new - r_old) / (r_old.z_old)
    sc->rz_old = sc->rz;
    sc->rz = tot[0];
    sc->rr = tot[1];
    sc->beta = (mode == FIN_FCG_UPDATE ? tot[0] - tot[2] : tot[0]) / sc->rz_old;
    sc->it = sc->it + 1;
    // the update kernel skipped this step when p.Ap <= 0 (see k_cg_update);
    // r.z <= 0 would make the next step length meaningless: both end the solve
    // at the last iterate, as does a non-finite residual
    sc->done = (tot[1] <= sc->tol2 || sc->it >= sc->max_it || !(tot[1] == tot[1]) || !(sc->pq > 0.0) ||
                !(tot[0] > 0.0))
                   ? 1
                   : 0;
  }
  if (flag_host && mode != FIN_STORE) {
    // vector stores with system scope into pinned host memory; visible to
    // the host once an event recorded after this kernel has completed
    __hip_atomic_store(&flag_host[1], sc->it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&flag_host[0], sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

inline unsigned grid_for(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// --- plain reductions
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sum(const T* x, int64_t n, double* partials, unsigned* counter,
                                                  double* out) {
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    v[0] += (double)x[i];
  block_partials<1>(v, partials);
}
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot(const T* x, const T* y, int64_t n, double* partials,
                                                  unsigned* counter, double* out) {
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    v[0] += (double)x[i] * (double)y[i];
  block_partials<1>(v, partials);
}

// y = x - sum/n (projection onto 1^T y = 0)
template <typename T>
__global__ void k_sub_mean(const T* x, T* y, int64_t n, const double* sum) {
  const double m = *sum / (double)n;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    y[i] = (T)((double)x[i] - m);
}

__global__ void k_clear_flag(int* f) { *f = 0; }
__global__ void k_phase(const double* phi, const double* prev, double* p64, float* p32, int64_t n, int* bad) {
  bool ok = true;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    double v = prev ? 0.5 * (phi[i] + prev[i]) : phi[i];
    ok = ok && __builtin_isfinite(v);
    p64[i] = v;
    // FP32 copy holds 1 + phi: near phi = -1 (the light phase) this keeps the
    // relative accuracy of rho = (beta - alpha) + alpha (1 + phi) at high
    // density ratios, where alpha phi + beta would cancel.
    p32[i] = (float)(1.0 + v);
  }
  // the pull back would map a NaN to a pure phase; flag it instead
  if (!ok) *bad = 1;
}

template <typename T>
__global__ void k_fill(T* x, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) x[i] = v;
}

__global__ void k_init_scalars(DevScalars* sc, double tol2, int max_it) {
  sc->tol2 = tol2;
  sc->max_it = max_it;
  sc->it = 0;
  sc->done = 0;
  sc->rz = sc->rr = sc->pq = sc->alpha = sc->beta = 0.0;
}

// --- CG kernels
// r = b - q; z = dinv r; p = z; rz, rr
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_init(const T* b, const T* q, T* r, T* z, T* p, const T* dinv,
                                                      int64_t n, DevScalars* sc, double* partials,
                                                      unsigned* counter) {
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    T ri = b[i] - q[i];
    T zi = dinv ? dinv[i] * ri : ri;
    r[i] = ri;
    z[i] = zi;
    if (p) p[i] = zi;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)ri * (double)ri;
  }
  block_partials<2>(v, partials);
}

// alpha = rz/pq; x += alpha p; r -= alpha q; z = dinv r; new rz, rr; beta
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_update(T* x, T* r, T* z, const T* p, const T* q, const T* dinv,
                                                        int64_t n, DevScalars* sc, double* partials,
                                                        unsigned* counter) {
  if (sc->done) return;
  // p.Ap <= 0 (breakdown of a non-SPD preconditioner, or p = 0): no step
  const double alpha = sc->pq > 0.0 ? sc->rz / sc->pq : 0.0;
  const T a = (T)alpha;
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    T xi = x[i] + a * p[i];
    T ri = r[i] - a * q[i];
    T zi = dinv ? dinv[i] * ri : ri;
    x[i] = xi;
    r[i] = ri;
    z[i] = zi;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)ri * (double)ri;
  }
  block_partials<2>(v, partials);
}

template <typename T>
__global__ void k_cg_p(T* p, const T* z, int64_t n, const DevScalars* sc, int check_done) {
  if (check_done && sc->done) return;
  const T beta = (T)sc->beta;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    p[i] = z[i] + beta * p[i];
}

// continued search direction after a residual replacement, in the units of
// the new inner system (right-hand side r / |r_new|; the previous one's was
// r / |r_old|, scale = |r_new| / |r_old|): CG p = z + scale (r.z) / rz_prev p;
// flexible CG (Polak-Ribiere) p = z + (scale (r.z) - z.r_prev) / rz_prev p
// with r_prev the previous inner system's last residual but one (z.r_prev in
// sc->beta) and rz_prev its r.z
template <typename T>
__global__ void k_cont_p(T* p, const T* z, int64_t n, const DevScalars* sc, double scale, double inv_rz_prev,
                         int flexible) {
  if (sc->done) return;
  const T beta = (T)((scale * sc->rz - (flexible ? sc->beta : 0.0)) * inv_rz_prev);
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    p[i] = z[i] + beta * p[i];
}

// r = b - q; partial r.r (slot 1)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_init_nopc(const T* b, const T* q, T* r, int64_t n,
                                                           double* partials) {
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    T ri = b[i] - q[i];
    r[i] = ri;
    v[1] += (double)ri * (double)ri;
  }
  block_partials<2>(v, partials);
}
// alpha = rz/pq; x += alpha p; (r_old = r); r -= alpha q; partial r.r (slot 1)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_update_nopc(T* x, T* r, T* r_old, const T* p, const T* q, int64_t n,
                                                             const DevScalars* sc, double* partials) {
  if (sc->done) return;
  const T a = (T)(sc->pq > 0.0 ? sc->rz / sc->pq : 0.0);
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const T ri = r[i];
    if (r_old) r_old[i] = ri;
    x[i] += a * p[i];
    const T rn = ri - a * q[i];
    r[i] = rn;
    v[1] += (double)rn * (double)rn;
  }
  block_partials<2>(v, partials);
}
// partial r.z (slot 0) and r_old.z (slot 2, flexible CG); slot 1 is left alone
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot_rz(const T* r, const T* z, const T* r_old, int64_t n,
                                                     const DevScalars* sc, double* partials, int respect_done) {
  __shared__ double sh[3][4];
  if (respect_done && sc->done) return;
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    a += (double)r[i] * (double)z[i];
    if (r_old) b += (double)r_old[i] * (double)z[i];
  }
  a = wsum(a);
  b = wsum(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = a;
    sh[2][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    partials[2 * kStride + blockIdx.x] = (sh[2][0] + sh[2][1]) + (sh[2][2] + sh[2][3]);
  }
}
template <typename T>
__global__ void k_copy(T* dst, const T* src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    dst[i] = src[i];
}

// x64 += scale * d32 ; r32 = (r64 - ...) handled separately
__global__ void k_ir_correct(double* x, const float* d, double scale, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    x[i] += scale * (double)d[i];
}
// r = b - q (FP64) and rr
__global__ __launch_bounds__(kThreads) void k_residual(const double* b, const double* q, double* r, int64_t n,
                                                       double* partials, unsigned* counter, double* out) {
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    double ri = b[i] - q[i];
    r[i] = ri;
    v[0] += ri * ri;
  }
  block_partials<1>(v, partials);
}
// r32 = r64 * s
__global__ void k_demote(const double* r, float* r32, double s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    r32[i] = (float)(r[i] * s);
}
__global__ void k_promote(const float* a, double* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    b[i] = (double)a[i];
}

int fin(Ctx& c, hipStream_t s, unsigned nparts, int nv, int mode, double* out, int respect_done) {
  k_finalize<<<1, kFinThreads, 0, s>>>(c.partials, (int)nparts, nv, mode, c.sc, out, respect_done, c.flag_host);
  CHNS_HIP(hipGetLastError());
  return CHNS_OK;
}

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

template <typename T>
T** work(Ctx& c);
template <>
double** work<double>(Ctx& c) {
  return c.w64;
}
template <>
float** work<float>(Ctx& c) {
  return c.w32;
}

template <typename T>
int ensure_work(Ctx& c, int k) {
  T** w = work<T>(c);
  if (!w[k]) w[k] = (T*)c.dalloc(sizeof(T) * c.dm.n * 3);
  return w[k] ? CHNS_OK : CHNS_ENOMEM;
}

int read_scalars(Ctx& c, hipStream_t s) {
  CHNS_HIP(hipMemcpyAsync(c.sc_host, c.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  CHNS_HIP(hipStreamSynchronize(s));
  return CHNS_OK;
}

// Host-side convergence polling that keeps the device busy: after each
// iteration an event is recorded; the host only waits for the iteration
// `depth - 1` behind the one it has just enqueued and then reads the done
// flag that the finaliser stores into pinned host memory (the value of that
// iteration or of a later one; done never returns to 0 within a solve).
// Iterations enqueued after convergence are no-ops for the CG kernels (they
// test the flag).
struct Poller {
  Ctx& c;
  hipStream_t s;
  int depth;
  std::vector<hipEvent_t> ev;
  Poller(Ctx& cc, hipStream_t ss, int d) : c(cc), s(ss), depth(d), ev(d, nullptr) {}
  ~Poller() {
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  int init() {
    for (auto& e : ev) CHNS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return CHNS_OK;
  }
  int post(int it) {
    CHNS_HIP(hipEventRecord(ev[it % depth], s));
    return CHNS_OK;
  }
  // wait for iteration `it` (already posted); true once the solve is done
  int wait(int it, bool* done) {
    CHNS_HIP(hipEventSynchronize(ev[it % depth]));
    *done = __atomic_load_n(&c.flag_host[0], __ATOMIC_ACQUIRE) != 0;
    return CHNS_OK;
  }
};

// PCK_JACOBI_FLEX: Jacobi applied between update and dot products (the
// flexible-CG form), for iterations that alternate with another preconditioner
enum PcKind { PCK_NONE = 0, PCK_JACOBI = 1, PCK_GMG = 2, PCK_LEARNED = 3, PCK_JACOBI_FLEX = 4 };
// iterations of flexible CG with the learned preconditioner before it is
// abandoned for Jacobi (stagnation guard)
constexpr int kLearnedCap = 400;

template <typename T>
__global__ void k_jacobi_pc(const T* d, const T* r, T* z, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    z[i] = d[i] * r[i];
}

template <typename T>
int apply_pc(Ctx& c, int pc, const T* r, T* z, hipStream_t s, const T* dinv = nullptr, int64_t n = 0) {
  if (pc == PCK_JACOBI_FLEX) {
    k_jacobi_pc<T><<<grid_for(n), kThreads, 0, s>>>(dinv, r, z, n);
    CHNS_HIP(hipGetLastError());
    return CHNS_OK;
  }
  if (pc == PCK_GMG) {
    if constexpr (sizeof(T) == 8) return mg_vcycle64(c, (const double*)r, (double*)z, s);
    else return mg_vcycle32(c, (const float*)r, (float*)z, s);
  }
  if (pc == PCK_LEARNED) return unet_apply<T>(c, r, z, s);
  set_error("unknown preconditioner");
  return CHNS_EINVAL;
}

// Preconditioned CG on A x = b with b in range(A) (1^T b = 0).  Vectors and
// the operator in precision T, dot products in FP64.  Jacobi (or none) is
// fused into the vector update; other preconditioners run between the update
// and the dot products.  flexible selects the Polak-Ribiere beta, which keeps
// CG convergent for a preconditioner that varies between iterations.  With
// every > 0 (flexible only) the preconditioner `pc` is applied to r_0 and
// after every `every`-th iteration, Jacobi after the others.
//
// cont_scale != 0 continues the search direction left in p (and, flexible,
// the residual left in r_old) by the previous call instead of starting from
// p = z (residual replacement, see the mixed solve); cont_scale is the ratio
// of the new to the previous normalisation of the right-hand side and
// cont_inv_rz the reciprocal of the previous call's last r.z but one; the
// schedule of `every` then counts on from sched_offset iterations.
template <typename T>
int pcg(Ctx& c, int op, const T* b, T* x, int pc, const T* dinv, bool flexible, double tol2, int max_it, int depth,
        bool graphs, hipStream_t s, int* iters, double* rr_out, int every = 0, double cont_scale = 0.0,
        double cont_inv_rz = 0.0, int sched_offset = 0) {
  // all fields of the operator form one vector (block-diagonal operators)
  const int64_t n = c.dm.n * op_fields(op, c.dm.dim);
  const int prec = sizeof(T) == 8 ? CHNS_FP64 : CHNS_FP32;
  for (int k = 0; k < 4; ++k)
    if (ensure_work<T>(c, k)) return CHNS_ENOMEM;
  if (flexible && ensure_work<T>(c, 6)) return CHNS_ENOMEM;
  T** w = work<T>(c);
  T *r = w[0], *z = w[1], *p = w[2], *q = w[3];
  T* r_old = flexible ? w[6] : nullptr;
  const bool fused_pc = pc == PCK_NONE || pc == PCK_JACOBI;
  const unsigned g = grid_for(n);
  Poller poll(c, s, std::max(1, depth));
  int rc = poll.init();
  if (rc) return rc;
  k_init_scalars<<<1, 1, 0, s>>>(c.sc, tol2, max_it);
  ApplyOut plain{};
  if ((rc = launch_apply(c, op, prec, x, q, s, plain))) return rc;
  const bool cont = cont_scale != 0.0;
  const bool cont_flex = cont && flexible && !fused_pc;
  if (fused_pc) {
    k_cg_init<T><<<g, kThreads, 0, s>>>(b, q, r, z, cont ? nullptr : p, pc == PCK_JACOBI ? dinv : nullptr, n, c.sc,
                                        c.partials, c.counter);
  } else {
    k_cg_init_nopc<T><<<g, kThreads, 0, s>>>(b, q, r, n, c.partials);
    // on a schedule, r_0 gets `pc` unless a continued solve is between turns
    const int pc0 = flexible && every > 0 && sched_offset % every != 0 ? PCK_JACOBI_FLEX : pc;
    if ((rc = apply_pc<T>(c, pc0, r, z, s, dinv, n))) return rc;
    k_dot_rz<T><<<g, kThreads, 0, s>>>(r, z, cont_flex ? r_old : nullptr, n, c.sc, c.partials, 0);
    if (!cont) k_copy<T><<<g, kThreads, 0, s>>>(p, z, n);
  }
  CHNS_HIP(hipGetLastError());
  if ((rc = fin(c, s, g, cont_flex ? 3 : 2, cont_flex ? FIN_FCG_CONT : FIN_CG_INIT, nullptr, 0))) return rc;
  if (cont) {
    k_cont_p<T><<<g, kThreads, 0, s>>>(p, z, n, c.sc, cont_scale, cont_inv_rz, cont_flex ? 1 : 0);
    CHNS_HIP(hipGetLastError());
  }
  ApplyOut fused{};
  fused.fuse_dot = true;
  fused.done = &c.sc->done;
  auto iteration = [&](hipStream_t st, int pck) -> int {
    int e;
    if ((e = launch_apply(c, op, prec, p, q, st, fused))) return e;
    if (fused_pc) {
      k_cg_update<T><<<g, kThreads, 0, st>>>(x, r, z, p, q, pc == PCK_JACOBI ? dinv : nullptr, n, c.sc,
                                             c.partials, c.counter);
      if ((e = fin(c, st, g, 2, FIN_CG_UPDATE, nullptr, 1))) return e;
    } else {
      k_cg_update_nopc<T><<<g, kThreads, 0, st>>>(x, r, r_old, p, q, n, c.sc, c.partials);
      if ((e = apply_pc<T>(c, pck, r, z, st, dinv, n))) return e;
      k_dot_rz<T><<<g, kThreads, 0, st>>>(r, z, r_old, n, c.sc, c.partials, 1);
      if ((e = fin(c, st, g, flexible ? 3 : 2, flexible ? FIN_FCG_UPDATE : FIN_CG_UPDATE, nullptr, 1))) return e;
    }
    k_cg_p<T><<<g, kThreads, 0, st>>>(p, z, n, c.sc, 1);
    CHNS_HIP(hipGetLastError());
    return CHNS_OK;
  };
  // one HIP graph per (operator, precision, preconditioner, variant, solution
  // and diagonal buffers); work buffers are context-owned, so the graph stays
  // valid across solves
  auto get_graph = [&](int pck, hipGraphExec_t* out) -> int {
    *out = nullptr;
    if (!graphs || c.prof) return CHNS_OK;
    for (auto& ge : c.graphs)
      if (ge.prec == prec && ge.pc == pck && ge.flexible == (int)flexible && ge.op == op &&
          ge.x == (const void*)x && ge.dinv == (const void*)dinv)
        *out = ge.exec;
    if (*out) return CHNS_OK;
    hipGraph_t graph = nullptr;
    hipGraphExec_t ex = nullptr;
    CHNS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    int e = iteration(s, pck);
    hipError_t ce = hipStreamEndCapture(s, &graph);
    if (e) return e;
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
    c.graphs.push_back({prec, pck, (int)flexible, op, (const void*)x, (const void*)dinv, ex});
    *out = ex;
    return CHNS_OK;
  };
  const bool sched = flexible && every > 0 && !fused_pc;
  hipGraphExec_t exec = nullptr, exec_j = nullptr;
  if ((rc = get_graph(pc, &exec))) return rc;
  if (sched && (rc = get_graph(PCK_JACOBI_FLEX, &exec_j))) return rc;
  bool done = false;
  int it = 0;
  while (true) {
    const bool jac = sched && (sched_offset + it + 1) % every != 0;
    hipGraphExec_t ex = jac ? exec_j : exec;
    if (ex) {
      CHNS_HIP(hipGraphLaunch(ex, s));
    } else if ((rc = iteration(s, jac ? PCK_JACOBI_FLEX : pc))) {
      return rc;
    }
    if ((rc = poll.post(it))) return rc;
    ++it;
    if (it >= max_it) break;
    if (it >= depth) {
      if ((rc = poll.wait(it - depth, &done))) return rc;
      if (done) break;
    }
  }
  CHNS_HIP(hipStreamSynchronize(s));
  if ((rc = read_scalars(c, s))) return rc;
  *iters = c.sc_host->it;
  *rr_out = c.sc_host->rr;
  return CHNS_OK;
}

}  // namespace

int launch_set_phase(Ctx& c, const double* phi, const double* prev, hipStream_t s) {
  k_clear_flag<<<1, 1, 0, s>>>(&c.sc->phi_bad);
  k_phase<<<grid_for(c.dm.n), kThreads, 0, s>>>(phi, prev, c.phi64, c.phi32, c.dm.n, &c.sc->phi_bad);
  CHNS_HIP(hipGetLastError());
  c.phi_set = true;
  c.diag_valid = false;
  if (c.mg) c.mg->setup_valid = false;
  return CHNS_OK;
}

int solve_pressure_impl(Ctx& c, const double* b_in, double* x_out, const chns_solve_opts& o,
                        chns_solve_stats& st, hipStream_t caller) {
  const int64_t n = c.dm.n;
  // work on the context stream after everything already queued on the caller's
  CHNS_HIP(hipEventRecord(c.ev_in, caller));
  CHNS_HIP(hipStreamWaitEvent(c.work, c.ev_in, 0));
  hipStream_t s = c.work;
  if (!c.xw64) c.xw64 = (double*)c.dalloc(sizeof(double) * n);
  if (!c.xw64) return CHNS_ENOMEM;
  double* x = c.xw64;
  CHNS_HIP(hipMemcpyAsync(x, x_out, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  const bool graphs = o.no_graphs == 0;
  const unsigned g = grid_for(n);
  if (!c.phi_set) {
    set_error("set_phase_field must be called before solve_pressure");
    return CHNS_ESTATE;
  }
  if (o.pc != CHNS_PC_JACOBI && o.pc != CHNS_PC_NONE && o.pc != CHNS_PC_GMG && o.pc != CHNS_PC_LEARNED) {
    set_error("unknown preconditioner");
    return CHNS_EINVAL;
  }
  const bool learned = o.pc == CHNS_PC_LEARNED;
  if (learned) {
    if (!unet_ready(c)) {
      set_error("no learned preconditioner weights in this context (chns_pc_load or chns_pc_init)");
      return CHNS_ESTATE;
    }
    int e = unet_prepare(c, s);
    if (e) return e;
  }
  int pck = o.pc == CHNS_PC_JACOBI ? PCK_JACOBI
                                   : (o.pc == CHNS_PC_GMG ? PCK_GMG : (learned ? PCK_LEARNED : PCK_NONE));
  // poll depth: cheap iterations can run far ahead, expensive ones not
  const int depth = (pck == PCK_GMG || learned) ? 2 : o.check_every;
  Timer t_setup;
  // projected right-hand side kept in w64[4]
  for (int k = 0; k < 6; ++k)
    if (ensure_work<double>(c, k)) return CHNS_ENOMEM;
  double* b = c.w64[4];
  double* sums = &c.sc->sum;
  int rc;
  k_sum<double><<<g, kThreads, 0, s>>>(b_in, n, c.partials, c.counter, sums);
  if ((rc = fin(c, s, g, 1, FIN_STORE, sums, 0))) return rc;
  k_sub_mean<double><<<g, kThreads, 0, s>>>(b_in, b, n, sums);
  k_dot<double><<<g, kThreads, 0, s>>>(b, b, n, c.partials, c.counter, &c.sc->bb);
  if ((rc = fin(c, s, g, 1, FIN_STORE, &c.sc->bb, 0))) return rc;
  CHNS_HIP(hipGetLastError());
  if (o.mode != CHNS_MODE_FP64 && o.mode != CHNS_MODE_MIXED_IR && o.mode != CHNS_MODE_MIXED_RU) {
    set_error("unknown solve mode");
    return CHNS_EINVAL;
  }
  const bool mixed = o.mode != CHNS_MODE_FP64;
  const bool replace = o.mode == CHNS_MODE_MIXED_RU;
  if (o.pc == CHNS_PC_GMG) {
    if ((rc = mg_build(c))) return rc;
    if (!c.mg->setup_valid && (rc = mg_setup(c, s))) return rc;
  }
  if (o.pc == CHNS_PC_JACOBI || learned) {
    // (the learned preconditioner falls back to Jacobi when it stagnates)
    if (!c.diag_valid) {
      if (!c.diag64) c.diag64 = (double*)c.dalloc(sizeof(double) * n);
      if (!c.diag32) c.diag32 = (float*)c.dalloc(sizeof(float) * n);
      if (!c.diag64 || !c.diag32) return CHNS_ENOMEM;
      for (int k = 6; k < 8; ++k) {
        if (!c.w64[k]) c.w64[k] = (double*)c.dalloc(sizeof(double) * n * 3);
        if (!c.w32[k]) c.w32[k] = (float*)c.dalloc(sizeof(float) * n * 3);
        if (!c.w64[k] || !c.w32[k]) return CHNS_ENOMEM;
      }
      auto diag_part = [&](hipStream_t st) -> int {
        int e = launch_diagonal(c, CHNS_OP_PRESSURE, CHNS_FP64, c.diag64, true, st);
        if (e) return e;
        return launch_diagonal(c, CHNS_OP_PRESSURE, CHNS_FP32, c.diag32, true, st);
      };
      if ((rc = graphs ? run_captured(c, &c.diag_exec, s, diag_part) : diag_part(s))) return rc;
      c.diag_valid = true;
    }
  }
  rc = read_scalars(c, s);
  if (rc) return rc;
  const double bb = c.sc_host->bb;
  st.ms_setup = t_setup.ms();
  Timer t_solve;
  st.iterations = 0;
  st.outer_iterations = 0;
  st.fallback = 0;
  if (c.sc_host->phi_bad) {
    st.rel_residual = NAN;
    st.ms_solve = 0.0;
    set_error("the phase field holds a NaN or an infinity");
    return CHNS_EINVAL;
  }
  if (!std::isfinite(bb)) {
    st.rel_residual = NAN;
    st.ms_solve = 0.0;
    set_error("the right-hand side holds a NaN or an infinity");
    return CHNS_EINVAL;
  }
  if (bb == 0.0) {
    k_fill<double><<<g, kThreads, 0, s>>>(x_out, 0.0, n);
    CHNS_HIP(hipStreamSynchronize(s));
    st.rel_residual = 0.0;
    st.ms_solve = t_solve.ms();
    return CHNS_OK;
  }
  const double tol2 = o.rtol * o.rtol * bb;
  double* q64 = c.w64[5];
  double* r64 = c.w64[0];
  ApplyOut plain{};
  if (!mixed) {
    int it = 0;
    double rr = 0;
    // learned every iteration: stagnation guard; on a schedule the Jacobi
    // iterations in between keep CG convergent
    const int every = learned ? o.learned_every : 0;
    const int cap = learned && every == 0 ? std::min(o.max_it, kLearnedCap) : o.max_it;
    rc = pcg<double>(c, CHNS_OP_PRESSURE, b, x, pck, c.diag64, learned, tol2, cap, every > 0 ? o.check_every : depth,
                     graphs, s, &it, &rr, every);
    if (rc) return rc;
    st.iterations = it;
    st.outer_iterations = 1;
    if (learned && !(rr <= tol2) && o.max_it > it) {
      // stagnation guard: continue from the current iterate with Jacobi-PCG
      st.fallback = 1;
      int it2 = 0;
      rc = pcg<double>(c, CHNS_OP_PRESSURE, b, x, PCK_JACOBI, c.diag64, false, tol2, o.max_it - it, o.check_every,
                       graphs, s, &it2, &rr);
      if (rc) return rc;
      st.iterations += it2;
    }
  } else {
    // FP64 iterative refinement: r = b - A x (FP64), inner FP32 CG on A d = r/|r|
    for (int k = 0; k < 5; ++k)
      if (ensure_work<float>(c, k)) return CHNS_ENOMEM;
    if (ensure_work<float>(c, 5)) return CHNS_ENOMEM;
    float* r32 = c.w32[4];
    float* d32 = c.w32[5];
    int total = 0;
    // residual replacement: the previous inner solve's |r| and its last
    // r.z before convergence (normalised units), for continuing its direction
    double rn_prev = 0.0, rz_prev = 0.0;
    bool can_continue = false;
    for (int outer = 0; outer < o.max_outer; ++outer) {
      rc = launch_apply(c, CHNS_OP_PRESSURE, CHNS_FP64, x, q64, s, plain);
      if (rc) return rc;
      k_residual<<<g, kThreads, 0, s>>>(b, q64, r64, n, c.partials, c.counter, &c.sc->rr);
      CHNS_HIP(hipGetLastError());
      if ((rc = fin(c, s, g, 1, FIN_STORE, &c.sc->rr, 0))) return rc;
      rc = read_scalars(c, s);
      if (rc) return rc;
      const double rr = c.sc_host->rr;
      st.outer_iterations = outer;
      if (rr <= tol2 || total >= o.max_it) break;
      const double rn = std::sqrt(rr);
      k_demote<<<g, kThreads, 0, s>>>(r64, r32, 1.0 / rn, n);
      // keep the inner right-hand side in range(A) after rounding
      k_sum<float><<<g, kThreads, 0, s>>>(r32, n, c.partials, c.counter, sums);
      if ((rc = fin(c, s, g, 1, FIN_STORE, sums, 0))) return rc;
      k_sub_mean<float><<<g, kThreads, 0, s>>>(r32, r32, n, sums);
      k_fill<float><<<g, kThreads, 0, s>>>(d32, 0.0f, n);
      CHNS_HIP(hipGetLastError());
      int it = 0;
      double rri = 0;
      const double itol = o.inner_rtol;
      const bool fcg = pck == PCK_LEARNED;
      const int every = fcg ? o.learned_every : 0;
      const int cap = fcg && every == 0 ? std::min(o.max_it - total, kLearnedCap) : o.max_it - total;
      // continued direction: this inner system is normalised by rn, the
      // previous one by rn_prev
      const bool cont = replace && can_continue;
      rc = pcg<float>(c, CHNS_OP_PRESSURE, r32, d32, pck, c.diag32, fcg, itol * itol, cap,
                      every > 0 ? o.check_every : depth, graphs, s, &it, &rri, every,
                      cont ? rn / rn_prev : 0.0, cont ? 1.0 / rz_prev : 0.0, cont ? total : 0);
      if (rc) return rc;
      total += it;
      rn_prev = rn;
      rz_prev = c.sc_host->rz_old;
      can_continue = it > 0 && rz_prev > 0.0 && std::isfinite(rz_prev);
      if (fcg && !(rri <= itol * itol)) {
        // stagnation guard: the remaining refinement steps use Jacobi
        st.fallback = 1;
        pck = PCK_JACOBI;
        can_continue = false;
      }
      k_ir_correct<<<g, kThreads, 0, s>>>(x, d32, rn, n);
      CHNS_HIP(hipGetLastError());
      st.outer_iterations = outer + 1;
    }
    st.iterations = total;
  }
  // x -> mean zero, then the FP64 true residual
  k_sum<double><<<g, kThreads, 0, s>>>(x, n, c.partials, c.counter, sums);
  if ((rc = fin(c, s, g, 1, FIN_STORE, sums, 0))) return rc;
  k_sub_mean<double><<<g, kThreads, 0, s>>>(x, x, n, sums);
  rc = launch_apply(c, CHNS_OP_PRESSURE, CHNS_FP64, x, q64, s, plain);
  if (rc) return rc;
  k_residual<<<g, kThreads, 0, s>>>(b, q64, r64, n, c.partials, c.counter, &c.sc->rr);
  CHNS_HIP(hipGetLastError());
  if ((rc = fin(c, s, g, 1, FIN_STORE, &c.sc->rr, 0))) return rc;
  CHNS_HIP(hipMemcpyAsync(x_out, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  rc = read_scalars(c, s);
  if (rc) return rc;
  st.rel_residual = std::sqrt(c.sc_host->rr / bb);
  st.ms_solve = t_solve.ms();
  if (!(st.rel_residual <= o.rtol)) {
    set_error("pressure solve did not reach rtol");
    return CHNS_ENOCONV;
  }
  return CHNS_OK;
}

int solve_spd_impl(Ctx& c, int op, const double* b, double* x, const double* dinv, double rtol, int max_it,
                   bool graphs, hipStream_t s, int* iters, double* rel) {
  const int64_t n = c.dm.n * op_fields(op, c.dm.dim);
  const unsigned g = grid_for(n);
  int rc;
  k_dot<double><<<g, kThreads, 0, s>>>(b, b, n, c.partials, c.counter, &c.sc->bb);
  if ((rc = fin(c, s, g, 1, FIN_STORE, &c.sc->bb, 0))) return rc;
  if ((rc = read_scalars(c, s))) return rc;
  const double bb = c.sc_host->bb;
  *iters = 0;
  *rel = 0.0;
  if (bb == 0.0) {
    k_fill<double><<<g, kThreads, 0, s>>>(x, 0.0, n);
    CHNS_HIP(hipGetLastError());
    return CHNS_OK;
  }
  double rr = 0.0;
  rc = pcg<double>(c, op, b, x, dinv ? PCK_JACOBI : PCK_NONE, dinv, false, rtol * rtol * bb, max_it, 16, graphs, s,
                   iters, &rr);
  if (rc) return rc;
  *rel = std::sqrt(rr / bb);
  if (!(*rel <= rtol)) {
    set_error("CG solve did not reach rtol");
    return CHNS_ENOCONV;
  }
  return CHNS_OK;
}

}  // namespace chns
