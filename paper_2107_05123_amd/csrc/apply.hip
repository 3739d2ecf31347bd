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
#include <algorithm>
#include <mutex>

#include "brick_geom.h"
#include "chns_internal.h"
#include "elem_chns.h"

namespace chns {
namespace {

// Slot buffer of the allocation-free apply (chns_apply_operator_noalloc):
// one per GPU, held until the process ends.  In host code `scratch` names a
// host-side stand-in; kernels get the device address from scratch_address().
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

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
// 1/sqrt(x) for x > 0: hardware estimate refined by two Newton steps
// y <- y + y (1 - x y^2) / 2 (FP64), the hardware value alone in FP32
__device__ __forceinline__ double rsqrt_t(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = __builtin_fma(-x * y, y, 1.0);
  y = __builtin_fma(0.5 * y, e, y);
  e = __builtin_fma(-x * y, y, 1.0);
  return __builtin_fma(0.5 * y, e, y);
}
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
// Pull back of the (scaled) phase field to its physical range.  FP64 fields
// hold phi in [-lim, lim]; FP32 fields hold 1 + phi in [0, 2 lim].
__device__ __forceinline__ double clamp_t(double v, double lim) { return fmin(fmax(v, -lim), lim); }
__device__ __forceinline__ float clamp_t(float v, float lim) { return __builtin_amdgcn_fmed3f(v, 0.0f, 2.0f * lim); }

// fused multiply-add in the operands' own precision (__builtin_fma is the
// double one: float operands would be widened and the result narrowed)
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// 1D two-node / two-Gauss-point transform, scaled by 2: (a, b) nodal values
// -> values at xi = -1/sqrt3, +1/sqrt3.  The 2x2 matrix is symmetric, so the
// same transform also applies the transpose.
template <typename T>
__device__ __forceinline__ void pair_tf(T& a, T& b) {
  T t = a + b;
  T u = b - a;
  a = fma_t(T(-kGauss), u, t);
  b = fma_t(T(kGauss), u, t);
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
template <int DIM, typename T, bool RCP = true>
__device__ __forceinline__ void elem_pp(const T* x, const T* ph, T A, T Bc, T* y) {
  constexpr int NC = 1 << DIM, H = NC / 2;
  T q[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) q[i] = ph[i];
  all_stages<DIM>(q);
  T c[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    // coefficient 1 / (A phi + B) (pressure) or A phi + B (viscosity)
    const T lin = fma_t(A, clamp_t(q[i], T(NC)), Bc);
    c[i] = RCP ? rcp_t(lin) : lin;
  }
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
    for (int i = 0; i < NC; ++i) r[i] = fma_t(A, clamp_t(r[i], T(NC)), Bc);
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
// NI gathered input fields (the vector x; wall nodes read as zero when
// MASK), NCF coefficient fields, NO output fields; WALL: 0 no special rows,
// 1 identity rows on the walls (y = x), 2 zero rows on the walls.
enum OpKind {
  K_PP = 0, K_MASS = 1, K_MASS_RHO = 2, K_CH_RES = 3, K_CH_JAC = 4, K_VP = 5, K_VP_RHS = 6, K_PP_RHS = 7,
  K_VU_RHS = 8, K_ENERGY = 9, K_PPS = 10, K_VPS = 11
};
template <int OP, int DIM>
struct Traits;
#define CHNS_TRAITS(OPK, ni, ncf, no, mask, wall)                  \
  template <int DIM>                                               \
  struct Traits<OPK, DIM> {                                        \
    static constexpr int NI = ni, NCF = ncf, NO = no, WALL = wall; \
    static constexpr bool MASK = mask;                             \
  };
CHNS_TRAITS(K_PP, 1, 1, 1, false, 0)
CHNS_TRAITS(K_MASS, 1, 0, 1, false, 0)
CHNS_TRAITS(K_MASS_RHO, DIM, 1, DIM, true, 1)
CHNS_TRAITS(K_CH_RES, 2, 2 + DIM, 2, false, 0)
CHNS_TRAITS(K_CH_JAC, 2, 1 + DIM, 2, false, 0)
CHNS_TRAITS(K_VP, DIM, 2 + DIM, DIM, true, 1)
CHNS_TRAITS(K_VP_RHS, 0, 3 * DIM + 3, DIM, false, 2)
CHNS_TRAITS(K_PP_RHS, 0, 4 * DIM + 3, 1, false, 0)
CHNS_TRAITS(K_VU_RHS, 0, 4 * DIM + 4, DIM, false, 2)
CHNS_TRAITS(K_ENERGY, 0, 2 + DIM, 1, false, 0)
CHNS_TRAITS(K_PPS, 1, 1, 1, false, 0)  // pressure operator + shift * mass
CHNS_TRAITS(K_VPS, 1, 1, 1, false, 0)  // scalar momentum: K_{eta/(2 Re)} + M_{rho/dt}
#undef CHNS_TRAITS

constexpr int kMaxCoef = kMaxCoefFields;

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
  const T* cf[kMaxCoef];  // coefficient fields (stride n each)
  T* y;
  T* slots;
  const int32_t* hang;
  const uint8_t* wall;
  double alpha, beta;  // rho(phi) = alpha phi + beta
  Phys phys;           // physical parameters of the CHNS forms
  double* partials;    // fused x.y partial per block, or null
  const int* done;
  // damped-Jacobi sweep (pressure operator): y = x + sm_w sm_d (sm_r - A x)
  const T* sm_r;
  const T* sm_d;
  T sm_w;
  double shift;  // K_PPS: mass shift
  // structured (uniform, lexicographically numbered) meshes: node indices are
  // computed from the brick anchor instead of read from the table
  const int32_t* anchor;  // 3 per brick, integer node coordinates
  int64_t sy, sz;         // index strides of y and z
  int32_t side;           // nodes per edge - 1
  // table meshes, 3D 8^3 bricks: eight block bases per brick (base[0] < 0:
  // use the table), from which the node numbers are computed
  const int32_t* abase;
};

// -------------------------------------------------- CHNS element routines
// (corner arrays as in elem_chns.h; w = det J, gs = 2/h)
template <int DIM>
__device__ __forceinline__ void el_ch_res(const double (*x)[1 << DIM], const double (*c)[1 << DIM], const Phys& P,
                                          double gs, double w, double (*y)[1 << DIM]) {
  constexpr int NC = 1 << DIM;
  double pt[NC], mt[NC], dp[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    pt[a] = 0.5 * (x[0][a] + c[0][a]);
    mt[a] = 0.5 * (x[1][a] + c[1][a]);
    dp[a] = x[0][a] - c[0][a];
    y[0][a] = 0.0;
    y[1][a] = 0.0;
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const double ptq = QP<DIM>::val(pt, q), dpq = QP<DIM>::val(dp, q), mtq = QP<DIM>::val(mt, q);
    double gpt[DIM], gmt[DIM], fl[DIM], fm[DIM];
    QP<DIM>::grad(pt, q, gs, gpt);
    QP<DIM>::grad(mt, q, gs, gmt);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double ut = QP<DIM>::val(c[2 + d], q);
      fl[d] = w * (-ut * ptq + gmt[d] / (P.Pe * P.Cn));
      fm[d] = w * P.Cn * P.Cn * gpt[d];
    }
    const double fphi = w * dpq / P.dt, fmu = w * (dpsi(ptq) - mtq);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      double s0 = refN<DIM>(q, a) * fphi, s1 = refN<DIM>(q, a) * fmu;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double gN = gs * refD<DIM>(q, a, d);
        s0 += gN * fl[d];
        s1 += gN * fm[d];
      }
      y[0][a] += s0;
      y[1][a] += s1;
    }
  }
}

// right-hand sides: coefficient layout phi~, mu~, u^ (DIM), u^k (DIM), p^k,
// then v (DIM) and p^{k+1}, and last the body force f_v (DIM; zero except for
// manufactured solutions), which is the known right-hand side of the momentum
// equation: (w, f_v) in the velocity prediction and -f_v inside R_m
template <int DIM>
__device__ __forceinline__ void el_vp_rhs(const double (*c)[1 << DIM], const Phys& P, double gs, double w,
                                          double (*y)[1 << DIM]) {
  constexpr int NC = 1 << DIM;
  const double* uh[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) uh[d] = c[2 + d];
  const double* pk = c[2 + 2 * DIM];
  constexpr int FV = 3 + 2 * DIM;  // first body-force row
#pragma unroll
  for (int f = 0; f < DIM; ++f)
#pragma unroll
    for (int a = 0; a < NC; ++a) y[f][a] = 0.0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    MomQ<DIM> M;
    M.init(P, c[0], c[1], uh, q, gs);
    double gp[DIM];
    QP<DIM>::grad(pk, q, gs, gp);
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      const double* uk = c[2 + DIM + i];
      const double ui = QP<DIM>::val(uk, q);
      double gui[DIM];
      QP<DIM>::grad(uk, q, gs, gui);
      const double kort = kort_i<DIM>(c[0], q, i, gs, M.gphi);
      const double fvi = QP<DIM>::val(c[FV + i], q);
      const double rk = M.rknown(P, i, ui, gui, gp, kort) - fvi;
      const double g = i == P.gaxis ? -1.0 : 0.0;
      const double fN = w * (M.rho * ui / P.dt - 0.5 * M.rho * M.dot(M.uh, gui) - M.dot(M.J, gui) / (2.0 * P.Pe) -
                             gp[i] + M.rho * g / P.Fr + fvi);
      double fG[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) fG[d] = w * (-M.eta * gui[d] / (2.0 * P.Re) + P.Cn / P.We * M.gphi[i] * M.gphi[d]);
      const double fst = -w * M.tau * rk;
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        double gN[DIM];
        gradN<DIM>(q, a, gs, gN);
        y[i][a] += refN<DIM>(q, a) * fN + M.dot(gN, fG) + M.s(P, gN) * fst;
      }
    }
  }
}

template <int DIM>
__device__ __forceinline__ void el_pp_rhs(const double (*c)[1 << DIM], const Phys& P, double gs, double w,
                                          double (*y)[1 << DIM]) {
  constexpr int NC = 1 << DIM;
  const double* uh[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) uh[d] = c[2 + d];
  const double* pk = c[2 + 2 * DIM];
  constexpr int FV = 3 + 3 * DIM;  // first body-force row
#pragma unroll
  for (int a = 0; a < NC; ++a) y[0][a] = 0.0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    MomQ<DIM> M;
    M.init(P, c[0], c[1], uh, q, gs);
    double gp[DIM], fG[DIM];
    QP<DIM>::grad(pk, q, gs, gp);
    double div = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      const double* v = c[3 + 2 * DIM + i];
      const double* uk = c[2 + DIM + i];
      double gv[DIM], gui[DIM];
      QP<DIM>::grad(v, q, gs, gv);
      QP<DIM>::grad(uk, q, gs, gui);
      div += gv[i];
      const double rl = M.rlin(P, QP<DIM>::val(v, q), gv);
      const double rk = M.rknown(P, i, QP<DIM>::val(uk, q), gui, gp, kort_i<DIM>(c[0], q, i, gs, M.gphi)) -
                        QP<DIM>::val(c[FV + i], q);
      fG[i] = w * (-(2.0 / P.dt) * M.tau * (rl + rk) / M.rho + gp[i] / M.rho);
    }
    const double fN = -w * (2.0 / P.dt) * div;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      double gN[DIM];
      gradN<DIM>(q, a, gs, gN);
      y[0][a] += refN<DIM>(q, a) * fN + M.dot(gN, fG);
    }
  }
}

template <int DIM>
__device__ __forceinline__ void el_vu_rhs(const double (*c)[1 << DIM], const Phys& P, double gs, double w,
                                          double (*y)[1 << DIM]) {
  constexpr int NC = 1 << DIM;
  const double* uh[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) uh[d] = c[2 + d];
  const double* pk = c[2 + 2 * DIM];
  const double* pn = c[3 + 3 * DIM];
  constexpr int FV = 4 + 3 * DIM;  // first body-force row
#pragma unroll
  for (int f = 0; f < DIM; ++f)
#pragma unroll
    for (int a = 0; a < NC; ++a) y[f][a] = 0.0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    MomQ<DIM> M;
    M.init(P, c[0], c[1], uh, q, gs);
    double gp[DIM], gpn[DIM];
    QP<DIM>::grad(pk, q, gs, gp);
    QP<DIM>::grad(pn, q, gs, gpn);
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      const double* v = c[3 + 2 * DIM + i];
      const double* uk = c[2 + DIM + i];
      double gv[DIM], gui[DIM];
      QP<DIM>::grad(v, q, gs, gv);
      QP<DIM>::grad(uk, q, gs, gui);
      const double vq = QP<DIM>::val(v, q);
      const double rl = M.rlin(P, vq, gv);
      const double rk = M.rknown(P, i, QP<DIM>::val(uk, q), gui, gp, kort_i<DIM>(c[0], q, i, gs, M.gphi)) -
                        QP<DIM>::val(c[FV + i], q);
      const double f = w * (M.rho * vq - M.tau * (rl + rk) - 0.5 * P.dt * (gpn[i] - gp[i]));
#pragma unroll
      for (int a = 0; a < NC; ++a) y[i][a] += refN<DIM>(q, a) * f;
    }
  }
}

// energy density of the leaf, split equally over its corners:
// 1/2 rho |u|^2 + (psi + Cn^2/2 |grad phi|^2)/(Cn We) + rho y / Fr
// (coefficients: phi, the vertical coordinate, u)
template <int DIM>
__device__ __forceinline__ void el_energy(const double (*c)[1 << DIM], const Phys& P, double gs, double w,
                                          double (*y)[1 << DIM]) {
  constexpr int NC = 1 << DIM;
  double e = 0.0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const double ph = QP<DIM>::val(c[0], q);
    const double rho = P.alpha * pull_back(ph) + P.beta;
    double g[DIM];
    QP<DIM>::grad(c[0], q, gs, g);
    double uu = 0.0, gg = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double u = QP<DIM>::val(c[2 + d], q);
      uu += u * u;
      gg += g[d] * g[d];
    }
    e += w * (0.5 * rho * uu + (psi(ph) + 0.5 * P.Cn * P.Cn * gg) / (P.Cn * P.We) + rho * QP<DIM>::val(c[1], q) / P.Fr);
  }
#pragma unroll
  for (int a = 0; a < NC; ++a) y[0][a] = e / NC;
}

// ---------------------------------------- heavy forms, corners read on demand
// The Cahn-Hilliard Jacobian and the VMS momentum operator read many fields;
// their element routines take the corner values through an accessor cv(f, a)
// (field f, corner a) that reads the brick's LDS node layers, so that no
// field is held in registers longer than it is used.
//
// Phase-field storage: FP64 fields hold phi, FP32 fields hold 1 + phi (so
// that rho = (beta - alpha) + alpha (1 + phi) keeps its relative accuracy
// near phi = -1 at large density ratios); PhaseT gives the pull-back range
// and the mixture laws in the stored variable.
template <typename T>
struct PhaseT {
  T lo, hi;          // range of the stored variable (phi* in [-1, 1])
  T ra, rb, ea, eb;  // rho = ra s + rb, eta = ea s + eb with s the stored value
};
template <typename T>
__device__ __forceinline__ PhaseT<T> phase_of(const Phys& P) {
  PhaseT<T> f;
  const bool shifted = sizeof(T) == 4;
  f.lo = shifted ? T(0) : T(-1);
  f.hi = shifted ? T(2) : T(1);
  f.ra = T(P.alpha);
  f.rb = T(shifted ? P.beta - P.alpha : P.beta);
  f.ea = T(P.gam);
  f.eb = T(shifted ? P.xi - P.gam : P.xi);
  return f;
}

// Newton Jacobian of the discrete Cahn-Hilliard system (Def. 6), fields
// x = [dphi, dmu] and coefficients [phi~ = (phi^{k+1} + phi^k)/2, u~]:
//   y_phi = M dphi / dt - 1/2 (grad q, u~ dphi) + K dmu / (2 Pe Cn)
//   y_mu  = 1/2 (q, psi''(phi~) dphi) + Cn^2/2 K dphi - 1/2 M dmu
// sum-factorised: values at the Gauss points by the two-point transforms,
// the constant-coefficient stiffness K in closed form (3D: the Q1 element
// matrix is (h/12)(5 I - 1 1^T + edge adjacency); 2D: (4 I - edge adjacency
// - 2 opposite corner)/6), the advection flux through the transposed
// gradient.  cv(f, a): f = 0 dphi, 1 dmu, 2 phi~, 3.. u~.
template <int DIM, typename T, class CV>
__device__ __forceinline__ void el_chj(const CV& cv, const Phys& P, int lev, T (*y)[1 << DIM]) {
  constexpr int NC = 1 << DIM, H = NC / 2;
  const double h = ldexp(1.0, -lev);
  // (2^d scaling of each transform) x (2^d of the transpose) folded into w
  const T w = T(ldexp(1.0, -(lev + 1) * DIM - 2 * DIM));
  const T inv2d = T(ldexp(1.0, -DIM));
  // stiffness parts, corner form
  {
    T xp[NC], xm[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      xp[a] = cv(0, a);
      xm[a] = cv(1, a);
    }
    const T kphi = T((DIM == 3 ? h / 12.0 : 1.0 / 6.0) * P.Cn * P.Cn * 0.5);
    const T kmu = T((DIM == 3 ? h / 12.0 : 1.0 / 6.0) / (2.0 * P.Pe * P.Cn));
    T sp = T(0), sm = T(0);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      sp += xp[a];
      sm += xm[a];
    }
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      T kp, km;
      if constexpr (DIM == 3) {
        kp = T(5) * xp[a] - sp + (xp[a ^ 1] + xp[a ^ 2] + xp[a ^ 4]);
        km = T(5) * xm[a] - sm + (xm[a ^ 1] + xm[a ^ 2] + xm[a ^ 4]);
      } else {
        kp = T(4) * xp[a] - (xp[a ^ 1] + xp[a ^ 2]) - T(2) * xp[a ^ 3];
        km = T(4) * xm[a] - (xm[a ^ 1] + xm[a ^ 2]) - T(2) * xm[a ^ 3];
      }
      y[0][a] = kmu * km;
      y[1][a] = kphi * kp;
    }
    // mass parts at the Gauss points (values scaled by 2^d)
    all_stages<DIM>(xp);
    all_stages<DIM>(xm);
    T pt[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) pt[a] = cv(2, a);
    all_stages<DIM>(pt);
    T fa[NC], fb[NC];
    const T idt = T(1.0 / P.dt);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const T p = pt[q] * inv2d;
      const T d2 = T(3) * p * p - T(1);
      fa[q] = w * idt * xp[q];
      fb[q] = w * T(0.5) * (d2 * xp[q] - xm[q]);
    }
    all_stages<DIM>(fa);
    all_stages<DIM>(fb);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      y[0][a] += fa[a];
      y[1][a] += fb[a];
    }
    // advection -1/2 (grad q, u~ dphi): flux F_d = -1/2 det J u~_d dphi at
    // each Gauss point, then the transposed gradient (constant along d)
    const T wa = T(-0.5 * ldexp(1.0, -(lev + 1) * DIM) * ldexp(1.0, lev) * ldexp(1.0, -2 * DIM - (DIM - 1)));
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      T u[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) u[a] = cv(3 + d, a);
      all_stages<DIM>(u);
      T g[H];
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const int lo = insert0(r, d), hi = lo | (1 << d);
        g[r] = u[lo] * xp[lo] + u[hi] * xp[hi];
      }
      stage<H, 1>(g);
      if constexpr (H > 2) stage<H, 2>(g);
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const int lo = insert0(r, d), hi = lo | (1 << d);
        const T v = wa * g[r];
        y[0][hi] += v;
        y[0][lo] -= v;
      }
    }
  }
}

// VMS velocity prediction (Def. 3, tau_m and R_m of Sec. 3.1), the same
// scalar operator for every component.  Per Gauss point, with
// b = u^/2 + J/(2 Pe rho~), g = grad eta~/(2 Re) and k = eta~/(2 Re):
//   R_lin(v) = rho~ (v/dt + b.grad v) - g.grad v,
//   Galerkin part  N_a rho~ (v/dt + b.grad v) + k grad N_a . grad v,
//   stabilisation  (b.grad N_a) tau_m R_lin(v).
// Sum-factorised: every field's values at the Gauss points come from the
// two-point transforms (scaled by S = 2^d), its gradient along d from the
// differences along d carried through the transforms of the other
// directions (constant along d, so shared by the two Gauss points of a
// column); the test functions are applied by the same transforms
// transposed.  The coefficients are formed once per Gauss point (the phase
// field clamped, tau_m, b scaled by 2/h, grad phi~ per column with the
// pull-back mask per point), then each component is transformed, combined
// and handed to out(f, y) in turn.  cv(f, a): f < DIM the velocity
// components, then phi~ (stored as in PhaseT), mu~, u^.
template <int DIM, typename T, class CV, class OUT>
__device__ __forceinline__ void el_vp(const CV& cv, const Phys& P, int lev, const OUT& out) {
  constexpr int NC = 1 << DIM, H = NC / 2;
  const PhaseT<T> ph = phase_of<T>(P);
  // powers of two (2/h = 2^e1, det J = 2^-d e1, S = 2^d) are applied with
  // ldexp: exact, and no per-level constants held in registers
  const int e1 = lev + 1;
  const double iS = ldexp(1.0, -DIM);  // 1/S
  const T idt = T(1.0 / P.dt);
  // k (2/h)^2 = (ea s + eb) / (2 Re) (2/h)^2; grad eta~ / (2 Re) (2/h) per
  // transformed column; J / (2 Pe) per transformed column
  const T kea = T(P.gam / (2.0 * P.Re)), keb = T(ph.eb / (2.0 * P.Re));
  const T cgp = T(P.gam / (2.0 * P.Re) * iS);
  const T cJ = T(P.cJ * iS / (2.0 * P.Pe));
  const T tau_c = T(4.0 / (P.dt * P.dt));
  const T visc_c = T(P.C_I * DIM);
  const T ire = T(1.0 / P.Re);
  const T iSt = T(iS);

  // ---- coefficients at the Gauss points
  T sc[NC], tau[NC], bs[DIM][NC], gp[DIM][H];
  unsigned inside = 0;
  {
    T v[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) v[a] = cv(DIM, a);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const int lo = insert0(r, d), hi = lo | (1 << d);
        gp[d][r] = v[hi] - v[lo];
      }
      stage<H, 1>(gp[d]);
      if constexpr (H > 2) stage<H, 2>(gp[d]);
#pragma unroll
      for (int r = 0; r < H; ++r) gp[d][r] = ldexp(gp[d][r] * cgp, 2 * e1);
    }
    all_stages<DIM>(v);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const T s = v[q] * iSt;
      sc[q] = fmin(fmax(s, ph.lo), ph.hi);
      if (s > ph.lo && s < ph.hi) inside |= 1u << q;
    }
  }
  asm volatile("" ::: "memory");
  {
    T J[DIM][H];
    {
      T m[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) m[a] = cv(DIM + 1, a);
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
#pragma unroll
        for (int r = 0; r < H; ++r) {
          const int lo = insert0(r, d), hi = lo | (1 << d);
          J[d][r] = m[hi] - m[lo];
        }
        stage<H, 1>(J[d]);
        if constexpr (H > 2) stage<H, 2>(J[d]);
#pragma unroll
        for (int r = 0; r < H; ++r) J[d][r] = ldexp(J[d][r] * cJ, e1);
      }
    }
    T irho[NC], uu[NC], uJ[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      irho[q] = rcp_t(ph.ra * sc[q] + ph.rb);
      uu[q] = uJ[q] = T(0);
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      asm volatile("" ::: "memory");
      T u[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) u[a] = cv(DIM + 2 + d, a);
      all_stages<DIM>(u);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int r = (q & ((1 << d) - 1)) | ((q >> (d + 1)) << d);
        const T uh = u[q] * iSt;
        const T j2 = J[d][r];  // J / (2 Pe)
        uu[q] = fma_t(uh, uh, uu[q]);
        uJ[q] = fma_t(uh, j2, uJ[q]);
        bs[d][q] = ldexp(fma_t(j2, irho[q], T(0.5) * uh), e1);
      }
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const T r = (ph.ea * sc[q] + ph.eb) * irho[q] * ire;
      // u^.J / (Pe rho~) = 2 u^.(J / (2 Pe)) / rho~
      tau[q] = rsqrt_t(tau_c + ldexp(fma_t(T(2) * uJ[q], irho[q], uu[q]), 2 * e1) + ldexp(visc_c * r * r, 4 * e1));
    }
  }
  // ---- the components in turn
#pragma unroll
  for (int f = 0; f < DIM; ++f) {
    asm volatile("" ::: "memory");
    T v[NC], g[DIM][H], fs[DIM][H];
#pragma unroll
    for (int a = 0; a < NC; ++a) v[a] = cv(f, a);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const int lo = insert0(r, d), hi = lo | (1 << d);
        g[d][r] = v[hi] - v[lo];
        fs[d][r] = T(0);
      }
      stage<H, 1>(g[d]);
      if constexpr (H > 2) stage<H, 2>(g[d]);
    }
    all_stages<DIM>(v);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const T rho = ph.ra * sc[q] + ph.rb;
      const T kg = ldexp(fma_t(kea, sc[q], keb), 2 * e1);
      T Gh = idt * v[q], gg = T(0);
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int r = (q & ((1 << d) - 1)) | ((q >> (d + 1)) << d);
        Gh = fma_t(bs[d][q], g[d][r], Gh);
        gg = fma_t(gp[d][r], g[d][r], gg);
      }
      const T A = rho * Gh;
      const T Tq = tau[q] * (((inside >> q) & 1u) ? A - gg : A);
      v[q] = A;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int r = (q & ((1 << d) - 1)) | ((q >> (d + 1)) << d);
        fs[d][r] = fma_t(kg, g[d][r], fma_t(bs[d][q], Tq, fs[d][r]));
      }
    }
    all_stages<DIM>(v);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      stage<H, 1>(fs[d]);
      if constexpr (H > 2) stage<H, 2>(fs[d]);
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const int lo = insert0(r, d), hi = lo | (1 << d);
        v[hi] += fs[d][r];
        v[lo] -= fs[d][r];
      }
    }
#pragma unroll
    for (int a = 0; a < NC; ++a) v[a] = ldexp(v[a], -(e1 + 2) * DIM);  // det J / S^2
    out(f, v);
  }
}

template <typename T, bool MASK>
__device__ __forceinline__ T fetch(const T* v, const uint8_t* wall, int32_t i) {
  if constexpr (MASK) return wall[i] ? T(0) : v[i];
  return v[i];
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The hardware deals workgroups round-robin to the 8 XCDs (block b runs on
// XCD b % 8), each with its own L2.  Bricks are numbered along the Morton
// curve, so handing XCD x the contiguous run of brick groups
// [start(x), start(x) + count(x)) keeps the node layers that neighbouring
// bricks share in one L2.  A bijection for any grid size.
__device__ __forceinline__ uint32_t xcd_block() {
  constexpr uint32_t kXcd = 8;
  const uint32_t g = gridDim.x, b = blockIdx.x;
  const uint32_t per = g / kXcd, rem = g % kXcd, x = b % kXcd;
  return x * per + (x < rem ? x : rem) + b / kXcd;
}

// One wavefront = BPB bricks; one lane = one leaf column of a brick, marching
// along the last axis.  WHOLE: every node of the brick is gathered into LDS
// up front (all loads in flight together); otherwise a three-layer LDS ring
// is refilled from registers two layers ahead.  STRUCT: uniform mesh with
// lexicographic node numbers, 32-bit offsets computed from the brick anchor.
// The layer march is unrolled for the small scalar forms (pressure, mass):
// ring slots, carries and node offsets become constants.
template <int DIM, int B, typename T, int OP, bool WHOLE, bool STRUCT>
__device__ __forceinline__ void brick_body(const BrickArgs<T>& a) {
  using TR = Traits<OP, DIM>;
  constexpr int NI = TR::NI, NCF = TR::NCF, NO = TR::NO, NV = NI + NCF;
  constexpr int NIa = NI > 0 ? NI : 1, NCa = NCF > 0 ? NCF : 1;
  constexpr int LPB = DIM == 3 ? B * B : B;  // lanes (leaf columns) per brick
  constexpr int BPB = 64 / LPB;              // bricks per wavefront
  constexpr int NL = DIM == 3 ? (B + 1) * (B + 1) : (B + 1);  // nodes per layer
  constexpr int KL = (NL + LPB - 1) / LPB;   // layer nodes handled per lane
  constexpr int NC = 1 << DIM, NH = NC / 2;
  // heavy forms read corners from LDS on demand; a two-layer ring suffices
  // for them (the layer two ahead is stored after the barrier that ends the
  // reads of the layer it replaces) and leaves LDS for two waves per SIMD
  constexpr bool HEAVY = OP == K_VP || OP == K_CH_JAC;
  constexpr int RING = WHOLE ? B + 1 : (HEAVY ? 2 : 3);
  __shared__ T lay[RING][BPB][NV][NL];
  // per-corner-type leaf contributions, indexed by the node they land on
  // (zero where no leaf of the brick lands): a node sums NH entries
  __shared__ T accn[BPB][NO][NH][NL];
  if (a.done && *a.done) return;
  const int lane = threadIdx.x, bl = lane / LPB, ll = lane % LPB;
  const int64_t brick = (int64_t)xcd_block() * BPB + bl;
  const bool active = brick < a.count;
  const int ix = ll % B, iy = DIM == 3 ? ll / B : 0;
  const int32_t* tab = a.table + (active ? brick : 0) * (int64_t)(NL * (B + 1));
  const int lev = active ? a.level[brick] : 0;
  int32_t base = 0;
  int32_t ax = 0, ay = 0, az = 0;
  if constexpr (STRUCT) {
    if (active) {
      ax = a.anchor[3 * brick];
      ay = a.anchor[3 * brick + 1];
      az = a.anchor[3 * brick + 2];
    }
    base = DIM == 3 ? ax + ay * (int32_t)a.sy + az * (int32_t)a.sz : ax + ay * (int32_t)a.sy;
  }
  // 8^3 bricks of a blocked node order whose numbers follow their 2x2x2
  // point blocks: node (jx, jy, z) is the base of its block plus its
  // lexicographic place in the block (the host checked this against the
  // table); the brick is one wavefront, so the choice is uniform.  Used by
  // the pressure and momentum forms only: in the others the extra registers
  // cost more (spills under the four-wave cap, a wave less for the CH
  // Jacobian) than the table loads they save
  constexpr bool AFF = !STRUCT && DIM == 3 && B == 8 && (OP == K_PP || OP == K_VP);
  int32_t ab[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool affine = false;
  if constexpr (AFF) {
    if (a.abase && active) {
      const int32_t* q = a.abase + brick * 8;
#pragma unroll
      for (int i = 0; i < 8; ++i) ab[i] = q[i];
      affine = ab[0] >= 0;
    }
  }
  auto affine_id = [&](int z, int p) -> int32_t {
    const int jx = p % (B + 1), jy = p / (B + 1);
    const bool zb = (z >> 3) != 0, yb = (jy >> 3) != 0, xb = (jx >> 3) != 0;
    const int32_t b0 = zb ? ab[4] : ab[0], b1 = zb ? ab[5] : ab[1], b2 = zb ? ab[6] : ab[2], b3 = zb ? ab[7] : ab[3];
    const int32_t bb = yb ? (xb ? b3 : b2) : (xb ? b1 : b0);
    return bb + (jx & 7) + 8 * (jy & 7) + 64 * (z & 7);
  };
  // index of layer-z node p (STRUCT) or its table entry
  auto entry = [&](int z, int p) -> int64_t {
    if constexpr (STRUCT) {
      const int jx = p % (B + 1), jy = DIM == 3 ? p / (B + 1) : 0;
      return DIM == 3 ? base + jx + jy * (int32_t)a.sy + z * (int32_t)a.sz : base + jx + z * (int32_t)a.sy;
    } else {
      if constexpr (AFF) {
        if (affine) return affine_id(z, p);
      }
      return tab[z * NL + p];
    }
  };
  auto on_wall = [&](int z, int p) -> bool {
    const int jx = p % (B + 1), jy = DIM == 3 ? p / (B + 1) : 0;
    const int cx = ax + jx, cy = DIM == 3 ? ay + jy : ay + z, cz = az + z;
    return cx == 0 || cx == a.side || cy == 0 || cy == a.side || (DIM == 3 && (cz == 0 || cz == a.side));
  };
  // structured meshes: field f of the node with index e at layer z, layer
  // position p (inputs read as zero on the walls when MASK)
  auto value = [&](int f, int64_t e, int z, int p) -> T {
    if (f < NI) {
      if constexpr (TR::MASK) {
        if (on_wall(z, p)) return T(0);
      }
      return (a.x + f * a.n)[(int32_t)e];
    }
    return a.cf[f - NI][(int32_t)e];
  };
  // Table meshes, every field of node entry e in two passes: first one load
  // per field with no branch (a hanging node reads node 0 as a placeholder),
  // so that all of them are in flight together; then, only in waves that
  // hold a hanging node, its fields replaced by the mean of its parents
  // (edge: (a + b) / 2, face: ((a + b) + (c + d)) / 4).
  auto table_vals = [&](int32_t e, T* v) {
    const int32_t i = e >= 0 ? e : 0;
#pragma unroll
    for (int f = 0; f < NV; ++f) v[f] = f < NI ? fetch<T, TR::MASK>(a.x + f * a.n, a.wall, i) : a.cf[f - NI][i];
  };
  auto table_hang = [&](int32_t e, T* v) {
    const int32_t* hp = a.hang + 4 * (int64_t)(-e - 1);
    const int32_t p0 = hp[0], p1 = hp[1], p2 = hp[2], p3 = hp[3];
    const bool four = p2 >= 0;
    const int32_t q2 = four ? p2 : p0, q3 = four ? p3 : p1;
#pragma unroll
    for (int f = 0; f < NV; ++f) {
      T v0, v1, v2, v3;
      if (f < NI) {
        const T* src = a.x + f * a.n;
        v0 = fetch<T, TR::MASK>(src, a.wall, p0);
        v1 = fetch<T, TR::MASK>(src, a.wall, p1);
        v2 = fetch<T, TR::MASK>(src, a.wall, q2);
        v3 = fetch<T, TR::MASK>(src, a.wall, q3);
      } else {
        const T* src = a.cf[f - NI];
        v0 = src[p0];
        v1 = src[p1];
        v2 = src[q2];
        v3 = src[q3];
      }
      const T s01 = v0 + v1;
      v[f] = four ? (s01 + (v2 + v3)) * T(0.25) : s01 * T(0.5);
    }
  };
  // per-level folded constants (powers of two are exact); FP32 fields carry
  // 1 + phi, so rho = (beta - alpha) + alpha (1 + phi)
  const double beta0 = sizeof(T) == 8 ? a.beta : a.beta - a.alpha;
  T A = 0, Bc = 0, Ms = 0, Am = 0, Bm = 0;
  if constexpr (OP == K_PPS) Ms = T(a.shift * ldexp(1.0, -(lev + 1) * DIM - 2 * DIM));
  if constexpr (OP == K_VPS) {
    // viscosity eta/(2 Re) = (gam phi + xi)/(2 Re) on the stiffness (folded
    // like the pressure coefficient, without the reciprocal) and rho/dt on
    // the mass
    const int es = (lev + 1) * (DIM - 2) + 2 * DIM, em = -(lev + 1) * DIM - 2 * DIM;
    const double g2 = a.phys.gam / (2.0 * a.phys.Re), x2 = a.phys.xi / (2.0 * a.phys.Re);
    A = T(ldexp(g2, -es - DIM));
    Bc = T(ldexp(sizeof(T) == 8 ? x2 : x2 - g2, -es));
    Am = T(ldexp(a.alpha / a.phys.dt, em - DIM));
    Bm = T(ldexp(beta0 / a.phys.dt, em));
  }
  if constexpr (OP == K_PP || OP == K_PPS) {
    // c~ = detJ (2/h)^2 / 4^d / rho = 1 / (rho / K); K = 2^{-(lev+1)(d-2) - 2d}
    const int e = (lev + 1) * (DIM - 2) + 2 * DIM;
    A = T(ldexp(a.alpha, e - DIM));
    Bc = T(ldexp(beta0, e));
  } else if constexpr (OP == K_MASS) {
    Bc = T(ldexp(1.0, -(lev + 1) * DIM - 2 * DIM));
  } else if constexpr (OP == K_MASS_RHO) {
    const int e = -(lev + 1) * DIM - 2 * DIM;
    A = T(ldexp(a.alpha, e - DIM));
    Bc = T(ldexp(beta0, e));
  }
  // CHNS forms: physical gradient scale 2/h and det J = (h/2)^d
  const double gs = ldexp(1.0, lev + 1), wdet = ldexp(1.0, -(lev + 1) * DIM);

  // -------- layered pipeline state (entries three layers ahead, values two)
  int64_t ent[KL];
  T val[KL][NV];
  // table meshes read the node entries one layer ahead of the values;
  // structured meshes compute them where they are used
  auto load_entries = [&](int z) {
    if constexpr (!STRUCT) {
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int p = ll + k * LPB;
        ent[k] = (active && z <= B && p < NL) ? entry(z, p) : 0;
      }
    }
  };
  auto gather_vals = [&](int z) {
    if constexpr (STRUCT) {
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int p = ll + k * LPB;
        if (active && z <= B && p < NL) {
          const int64_t e = entry(z, p);
#pragma unroll
          for (int f = 0; f < NV; ++f) val[k][f] = value(f, e, z, p);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int p = ll + k * LPB;
        if (active && z <= B && p < NL) table_vals((int32_t)ent[k], val[k]);
      }
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int p = ll + k * LPB;
        if (active && z <= B && p < NL && ent[k] < 0) table_hang((int32_t)ent[k], val[k]);
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
        eo[k] = (active && p < NL) ? entry(z, p) : 0;
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
      T v[NO];
#pragma unroll
      for (int f = 0; f < NO; ++f) {
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
        if constexpr (OP == K_PP || OP == K_PPS || OP == K_VPS) {
          if (a.sm_r) v[0] = lay[buf][bl][0][p] + a.sm_w * a.sm_d[e] * (a.sm_r[e] - v[0]);
        }
#pragma unroll
        for (int f = 0; f < NO; ++f) {
          a.y[f * a.n + e] = v[f];
          if constexpr (NI == NO && !HEAVY) {
            if (a.partials) dot += (double)lay[buf][bl][f][p] * (double)v[f];
          }
        }
      } else {
        const int64_t sl = a.slot_base + brick * a.nbnd + brick_rank(DIM, B, jx, jy, z);
#pragma unroll
        for (int f = 0; f < NO; ++f) a.slots[f * a.n_slots + sl] = v[f];
      }
    }
  };

  T carry[NO][NH];
#pragma unroll
  for (int f = 0; f < NO; ++f)
#pragma unroll
    for (int c = 0; c < NH; ++c) carry[f][c] = T(0);

  if (active) {
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int p = ll + k * LPB;
      if (p < NL)
#pragma unroll
        for (int f = 0; f < NO; ++f)
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
      if constexpr (STRUCT) {
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
      } else {
        int32_t ew[KW];
#pragma unroll
        for (int k = 0; k < KW; ++k) {
          const int q = ll + k * LPB;
          ew[k] = q < NPB ? tab[q] : 0;
        }
#pragma unroll
        for (int k = 0; k < KW; ++k)
          if (ll + k * LPB < NPB) table_vals(ew[k], w[k]);
#pragma unroll
        for (int k = 0; k < KW; ++k)
          if (ll + k * LPB < NPB && ew[k] < 0) table_hang(ew[k], w[k]);
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
  T xc[NIa][NC], cc[NCa][NC];
  auto read_half = [&](int z, int half) {
#pragma unroll
    for (int c = 0; c < NH; ++c) {
      const int bx = c & 1, by = DIM == 3 ? (c >> 1) & 1 : 0;
      const int p = (ix + bx) + (DIM == 3 ? (iy + by) * (B + 1) : 0);
      const int buf = z % RING;
#pragma unroll
      for (int f = 0; f < NI; ++f) xc[f][c + half * NH] = lay[buf][bl][f][p];
#pragma unroll
      for (int f = 0; f < NCF; ++f) cc[f][c + half * NH] = lay[buf][bl][NI + f][p];
    }
  };
  if constexpr (!HEAVY) {
    if (active) read_half(0, 1);
  }
  constexpr int kUnroll = (OP == K_PP || OP == K_PPS || OP == K_VPS || OP == K_MASS) ? B : 1;
#pragma unroll kUnroll
  for (int ez = 0; ez < B; ++ez) {
    load_emit_entries(ez);
    if (active) {
      T ye[NO][NC];
      if constexpr (!HEAVY) {
#pragma unroll
        for (int c = 0; c < NH; ++c) {
#pragma unroll
          for (int f = 0; f < NI; ++f) xc[f][c] = xc[f][c + NH];
#pragma unroll
          for (int f = 0; f < NCF; ++f) cc[f][c] = cc[f][c + NH];
        }
        read_half(ez + 1, 1);
      }
      // corner a of field f (inputs first, then coefficients) from LDS
      auto cv = [&](int f, int ca) -> T {
        const int bx = ca & 1, by = DIM == 3 ? (ca >> 1) & 1 : 0, bz = (ca >> (DIM - 1)) & 1;
        const int p = (ix + bx) + (DIM == 3 ? (iy + by) * (B + 1) : 0);
        return lay[(ez + bz) % RING][bl][f][p];
      };
      if constexpr (OP == K_CH_JAC) {
        el_chj<DIM, T>(cv, a.phys, lev, ye);
      } else if constexpr (OP == K_VP) {
        // each component's corner values go to the node accumulators as
        // soon as they are formed
        el_vp<DIM, T>(cv, a.phys, lev, [&](int f, const T* yf) {
#pragma unroll
          for (int c = 0; c < NH; ++c) {
            const int p = (ix + (c & 1)) + (DIM == 3 ? (iy + ((c >> 1) & 1)) * (B + 1) : 0);
            accn[bl][f][c][p] = yf[c] + carry[f][c];
            carry[f][c] = yf[c + NH];
          }
        });
      } else if constexpr (OP == K_PP || OP == K_PPS) {
        elem_pp<DIM, T>(xc[0], cc[0], A, Bc, ye[0]);
        if constexpr (OP == K_PPS) {
          T r[NC], ym[NC];
#pragma unroll
          for (int i = 0; i < NC; ++i) r[i] = Ms;
          elem_mass_apply<DIM, T>(xc[0], r, ym);
#pragma unroll
          for (int i = 0; i < NC; ++i) ye[0][i] += ym[i];
        }
      } else if constexpr (OP == K_VPS) {
        elem_pp<DIM, T, false>(xc[0], cc[0], A, Bc, ye[0]);
        T r[NC], ym[NC];
        elem_mass_coef<DIM, T, true>(cc[0], Am, Bm, r);
        elem_mass_apply<DIM, T>(xc[0], r, ym);
#pragma unroll
        for (int i = 0; i < NC; ++i) ye[0][i] += ym[i];
      } else if constexpr (OP == K_MASS || OP == K_MASS_RHO) {
        T r[NC];
        elem_mass_coef<DIM, T, OP == K_MASS_RHO>(cc[0], A, Bc, r);
#pragma unroll
        for (int f = 0; f < NI; ++f) elem_mass_apply<DIM, T>(xc[f], r, ye[f]);
      } else if constexpr (OP == K_CH_RES) {
        el_ch_res<DIM>(xc, cc, a.phys, gs, wdet, ye);
      } else if constexpr (OP == K_VP_RHS) {
        el_vp_rhs<DIM>(cc, a.phys, gs, wdet, ye);
      } else if constexpr (OP == K_PP_RHS) {
        el_pp_rhs<DIM>(cc, a.phys, gs, wdet, ye);
      } else if constexpr (OP == K_VU_RHS) {
        el_vu_rhs<DIM>(cc, a.phys, gs, wdet, ye);
      } else {
        el_energy<DIM>(cc, a.phys, gs, wdet, ye);
      }
      if constexpr (OP != K_VP) {
#pragma unroll
        for (int f = 0; f < NO; ++f)
#pragma unroll
          for (int c = 0; c < NH; ++c) {
            const int p = (ix + (c & 1)) + (DIM == 3 ? (iy + ((c >> 1) & 1)) * (B + 1) : 0);
            accn[bl][f][c][p] = ye[f][c] + carry[f][c];
            carry[f][c] = ye[f][c + NH];
          }
      }
    }
    __syncthreads();
    // values of layer ez + 2 (loads in flight since the previous layer) go to
    // LDS before this layer's outputs are stored: waiting for those loads
    // then does not also wait for the stores
    if constexpr (!WHOLE) store_vals(ez + 2);
    emit_layer(ez);
    if constexpr (!WHOLE) {
      gather_vals(ez + 3);
      load_entries(ez + 4);
    }
    __syncthreads();
  }
  load_emit_entries(B);
  if (active) {
#pragma unroll
    for (int f = 0; f < NO; ++f)
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

template <int DIM, int B, typename T, int OP, bool WHOLE, bool STRUCT>
__global__ __launch_bounds__(64) void k_brick(BrickArgs<T> a) {
  brick_body<DIM, B, T, OP, WHOLE, STRUCT>(a);
}
// the pressure and mass forms (at most 128 VGPRs in FP64): capped at four
// waves per SIMD, which keeps the FP32 instances from trading their latency
// hiding for occupancy
template <int DIM, int B, typename T, int OP, bool WHOLE, bool STRUCT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_brick_o4(BrickArgs<T> a) {
  brick_body<DIM, B, T, OP, WHOLE, STRUCT>(a);
}
// the FP64 3D Cahn-Hilliard Jacobian on structured 8^3 bricks: its LDS
// admits three waves per SIMD, which at 128^3 leaves a third of the bricks
// to a second, sparse round; held to two waves it runs two full rounds
// (0.095 -> 0.090 ms; equal at 256^3; on adaptive meshes three are faster)
template <int DIM, int B, typename T, int OP, bool WHOLE, bool STRUCT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_brick_o2(BrickArgs<T> a) {
  brick_body<DIM, B, T, OP, WHOLE, STRUCT>(a);
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

template <typename T, int NO, int WALL>
__global__ __launch_bounds__(256) void k_combine(const int32_t* __restrict__ node, const int32_t* __restrict__ ptr,
                                                 const uint32_t* __restrict__ ent, int64_t nrows,
                                                 const T* __restrict__ slots, int64_t n_slots, T* __restrict__ y,
                                                 const T* __restrict__ x, int64_t n, const uint8_t* __restrict__ wall,
                                                 double* partials, const int* done, const T* __restrict__ sm_r,
                                                 const T* __restrict__ sm_d, T sm_w) {
  __shared__ double sh[4];
  if (done && *done) return;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dot = 0.0;
  if (row < nrows) {
    const int32_t i = node[row];
    const int32_t k0 = ptr[row], k1 = ptr[row + 1];
    // a row's entries and then its slots are loaded CH at a time, every load
    // of a group in flight together (a row holds 2 to 8 entries, more only
    // next to hanging nodes); the sum keeps the entry order
    constexpr int CH = 8;
    T v[NO];
#pragma unroll
    for (int f = 0; f < NO; ++f) v[f] = T(0);
    for (int32_t kb = k0; kb < k1; kb += CH) {
      uint32_t e[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) e[j] = kb + j < k1 ? ent[kb + j] : 0u;
#pragma unroll
      for (int f = 0; f < NO; ++f) {
        T sv[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) sv[j] = kb + j < k1 ? slots[f * n_slots + (e[j] & 0x3fffffffu)] : T(0);
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          if (kb + j < k1) {
            const uint32_t code = e[j] >> 30;
            v[f] += code == 0 ? sv[j] : (code == 1 ? sv[j] * T(0.5) : sv[j] * T(0.25));
          }
        }
      }
    }
#pragma unroll
    for (int f = 0; f < NO; ++f) {
      T w = v[f];
      // wall rows: identity (WALL 1) or zero (WALL 2)
      if constexpr (WALL == 1) {
        if (wall[i]) w = x[f * n + i];
      } else if constexpr (WALL == 2) {
        if (wall[i]) w = T(0);
      }
      if (sm_r) w = x[i] + sm_w * sm_d[i] * (sm_r[i] - w);
      y[f * n + i] = w;
      if (partials) dot += (double)x[f * n + i] * (double)w;
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

// FP32 copy of coefficient fields; entries below `shifted` (the phase field
// of the momentum operator) are stored as 1 + value
__global__ void k_coef32(const double* src, float* dst, int64_t n, int64_t shifted) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)(i < shifted ? 1.0 + src[i] : src[i]);
}

// Diagonal probing helpers.
// x = indicator of colour c in field `field` (every field when field < 0)
template <typename T>
__global__ void k_indicator(T* x, const uint8_t* color, int c, int64_t n, int nf, int field) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T v = color[i] == c ? T(1) : T(0);
  for (int f = 0; f < nf; ++f) x[f * n + i] = (field < 0 || f == field) ? v : T(0);
}
template <typename T>
__global__ void k_take_diag(T* d, const T* y, const uint8_t* color, int c, int64_t n, int nf, int invert,
                            int field) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (color[i] != c) return;
  for (int f = 0; f < nf; ++f) {
    if (field >= 0 && f != field) continue;
    T v = y[f * n + i];
    d[f * n + i] = invert ? (v != T(0) ? T(1) / v : T(1)) : v;
  }
}
// column `field` of the nf x nf node blocks: blk[(g * nf + field) * n + i] = y_g,i
__global__ void k_take_block(double* blk, const double* y, const uint8_t* color, int c, int64_t n, int nf,
                             int field) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (color[i] != c) return;
  for (int g = 0; g < nf; ++g) blk[(g * nf + field) * n + i] = y[g * n + i];
}

template <int DIM, int B, typename T, int OP>
constexpr bool whole_fits() {
  using TR = Traits<OP, DIM>;
  constexpr int LPB = DIM == 3 ? B * B : B;
  constexpr int NL = DIM == 3 ? (B + 1) * (B + 1) : (B + 1);
  // deep bricks keep the three-layer ring (better occupancy, loads pipelined)
  return B <= 4 && (64 / LPB) * NL * (B + 1) * (TR::NI + TR::NCF) * (int)sizeof(T) <= 12 * 1024;
}

template <int DIM, int B, typename T, int OP, bool STRUCT>
void launch_one(int64_t grid, hipStream_t s, const BrickArgs<T>& a) {
  const dim3 g((unsigned)grid), blk(64);
  constexpr bool W = whole_fits<DIM, B, T, OP>();
  // the scalar momentum form (viscous stiffness and density mass together)
  // needs ~140 registers: capped at four waves it spilled (88 bytes per lane
  // on table bricks), uncapped it runs three without
  if constexpr (OP == K_PP || OP == K_PPS || OP == K_MASS)
    k_brick_o4<DIM, B, T, OP, W, STRUCT><<<g, blk, 0, s>>>(a);
  else if constexpr (OP == K_CH_JAC && DIM == 3 && B == 8 && STRUCT && sizeof(T) == 8)
    k_brick_o2<DIM, B, T, OP, W, STRUCT><<<g, blk, 0, s>>>(a);
  else k_brick<DIM, B, T, OP, W, STRUCT><<<g, blk, 0, s>>>(a);
}
template <int DIM, typename T, int OP, bool STRUCT>
void launch_b(int B, int64_t grid, hipStream_t s, const BrickArgs<T>& a) {
  switch (B) {
    case 8: launch_one<DIM, 8, T, OP, STRUCT>(grid, s, a); break;
    case 4: launch_one<DIM, 4, T, OP, STRUCT>(grid, s, a); break;
    case 2: launch_one<DIM, 2, T, OP, STRUCT>(grid, s, a); break;
    default: launch_one<DIM, 1, T, OP, STRUCT>(grid, s, a); break;
  }
}

template <int DIM, typename T, int OP>
int launch_bricks(const DevMesh& dm, BrickArgs<T> a, hipStream_t s, int& part_off) {
  for (int k = 0; k < kBrickClasses; ++k) {
    const DevBrickClass& bc = dm.cls[k];
    if (bc.count == 0) continue;
    a.table = bc.table;
    a.abase = bc.abase;
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

Phys phys_of(const chns_params& p) {
  Phys f{};
  f.dt = p.dt;
  f.Pe = p.Pe;
  f.Cn = p.Cn;
  f.We = p.We;
  f.Re = p.Re;
  f.Fr = p.Fr;
  f.C_I = p.C_I;
  f.alpha = (p.rho_plus - p.rho_minus) / (2.0 * p.rho_plus);
  f.beta = (p.rho_plus + p.rho_minus) / (2.0 * p.rho_plus);
  f.gam = (p.eta_plus - p.eta_minus) / (2.0 * p.eta_plus);
  f.xi = (p.eta_plus + p.eta_minus) / (2.0 * p.eta_plus);
  f.cJ = (p.rho_minus - p.rho_plus) / (2.0 * p.rho_plus * p.Cn);
  f.gaxis = p.gravity_axis;
  return f;
}

const char* op_tag(int op, bool fp64) {
  static const char* tags[12][2] = {{"pp_brick_fp64", "pp_brick_fp32"},
                                    {"mass_brick_fp64", "mass_brick_fp32"},
                                    {"massrho_brick_fp64", "massrho_brick_fp32"},
                                    {"chres_brick_fp64", "chres_brick_fp32"},
                                    {"chjac_brick_fp64", "chjac_brick_fp32"},
                                    {"vp_brick_fp64", "vp_brick_fp32"},
                                    {"vprhs_brick_fp64", "vprhs_brick_fp32"},
                                    {"pprhs_brick_fp64", "pprhs_brick_fp32"},
                                    {"vurhs_brick_fp64", "vurhs_brick_fp32"},
                                    {"energy_brick_fp64", "energy_brick_fp32"},
                                    {"pps_brick_fp64", "pps_brick_fp32"},
                                    {"vps_brick_fp64", "vps_brick_fp32"}};
  return tags[op][fp64 ? 0 : 1];
}

// cf: the op's NCF coefficient fields (each n long, device)
template <int DIM, typename T, int OP>
int apply_t(Ctx& c, const LevelView& L, const T* x, T* y, const T* const* cf, hipStream_t s, const ApplyOut& o) {
  using TR = Traits<OP, DIM>;
  static_assert(TR::NCF <= kMaxCoef, "too many coefficient fields");
  const DevMesh& dm = *L.dm;
  if (o.fuse_dot && (TR::NI != TR::NO || OP == K_VP || OP == K_CH_JAC)) {
    set_error("fused dot needs as many inputs as outputs and a scalar-form operator");
    return CHNS_EINVAL;
  }
  if (o.sm_r && ((OP != K_PP && OP != K_PPS && OP != K_VPS) || o.fuse_dot || x == y)) {
    set_error("a fused smoothing sweep needs the pressure operator, no fused dot and y distinct from x");
    return CHNS_EINVAL;
  }
  BrickArgs<T> a{};
  a.n = dm.n;
  a.n_slots = dm.n_slots;
  a.x = x;
  for (int k = 0; k < TR::NCF; ++k) a.cf[k] = cf[k];
  a.y = y;
  a.slots = (T*)L.slots;
  a.hang = dm.hang_par;
  a.wall = dm.wall;
  a.phys = phys_of(c.prm);
  a.alpha = a.phys.alpha;
  a.beta = a.phys.beta;
  a.partials = o.fuse_dot ? c.partials : nullptr;
  a.done = o.done;
  a.sm_r = (const T*)o.sm_r;
  a.sm_d = (const T*)o.sm_dinv;
  a.sm_w = (T)o.sm_w;
  a.shift = c.pp_shift;
  a.sy = dm.side + 1;
  a.sz = (int64_t)(dm.side + 1) * (dm.side + 1);
  a.side = dm.side;
  int part_off = 0;
  const char* tag = op_tag(OP, sizeof(T) == 8);
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
    k_combine<T, TR::NO, TR::WALL><<<dim3(g), dim3(256), 0, s>>>(
        dm.comb_node, dm.comb_ptr, dm.comb_ent, dm.n_comb, (const T*)L.slots, dm.n_slots, y, x, dm.n, dm.wall,
        o.fuse_dot ? c.partials + part_off : nullptr, o.done, (const T*)o.sm_r, (const T*)o.sm_dinv,
        (T)o.sm_w);
    CHNS_HIP(hipGetLastError());
    c.prof_end("combine", s, ev);
  }
  if (o.fuse_dot) {
    k_sum_partials<<<1, 1024, 0, s>>>(c.partials, total, &c.sc->pq, o.done);
    CHNS_HIP(hipGetLastError());
  }
  return CHNS_OK;
}

template <int OP, typename T>
int apply_d(Ctx& c, const LevelView& L, const T* x, T* y, const T* const* cf, hipStream_t s, const ApplyOut& o) {
  return L.dm->dim == 3 ? apply_t<3, T, OP>(c, L, x, y, cf, s, o) : apply_t<2, T, OP>(c, L, x, y, cf, s, o);
}

template <typename T>
int apply_dispatch(Ctx& c, const LevelView& L, int op, const T* x, T* y, const T* phi, hipStream_t s,
                   const ApplyOut& o) {
  const T* one[1] = {phi};
  switch (op) {
    case CHNS_OP_PRESSURE:
      if (c.pp_kind == 1) return apply_d<K_VPS, T>(c, L, x, y, one, s, o);
      if (c.pp_shift != 0.0) return apply_d<K_PPS, T>(c, L, x, y, one, s, o);
      return apply_d<K_PP, T>(c, L, x, y, one, s, o);
    case CHNS_OP_MASS:
      return apply_d<K_MASS, T>(c, L, x, y, one, s, o);
    case CHNS_OP_MASS_RHO:
      return apply_d<K_MASS_RHO, T>(c, L, x, y, one, s, o);
    case CHNS_OP_MOMENTUM_SCALAR:
      return apply_d<K_VPS, T>(c, L, x, y, one, s, o);
  }
  if constexpr (sizeof(T) == 8) {
    const int64_t n = L.dm->n;
    const double* cf[kMaxCoef] = {};
    if (op == CHNS_OP_MOMENTUM || op == CHNS_OP_CH_JACOBIAN) {
      const bool mom = op == CHNS_OP_MOMENTUM;
      const double* base = mom ? c.coef_mom : c.coef_chj;
      if (!base || !(mom ? c.coef_mom_set : c.coef_chj_set)) {
        set_error("chns_set_coefficients must be called for this operator first");
        return CHNS_ESTATE;
      }
      for (int k = 0; k < (mom ? 2 : 1) + L.dm->dim; ++k) cf[k] = base + k * n;
      return mom ? apply_d<K_VP, double>(c, L, x, y, cf, s, o) : apply_d<K_CH_JAC, double>(c, L, x, y, cf, s, o);
    }
  } else {
    if (op == CHNS_OP_MOMENTUM || op == CHNS_OP_CH_JACOBIAN) {
      const bool mom = op == CHNS_OP_MOMENTUM;
      const double* base = mom ? c.coef_mom : c.coef_chj;
      if (!base || !(mom ? c.coef_mom_set : c.coef_chj_set)) {
        set_error("chns_set_coefficients must be called for this operator first");
        return CHNS_ESTATE;
      }
      // FP32 copies of the coefficient fields, refreshed after every change
      // of the FP64 ones (the momentum phase field as 1 + phi)
      const int64_t n = L.dm->n;
      const int nf = (mom ? 2 : 1) + L.dm->dim;
      float*& c32 = mom ? c.coef_mom32 : c.coef_chj32;
      bool& ok = mom ? c.coef_mom32_ok : c.coef_chj32_ok;
      if (!c32 && !(c32 = (float*)c.dalloc(sizeof(float) * (size_t)nf * (size_t)n))) return CHNS_ENOMEM;
      if (!ok) {
        const int64_t tot = nf * n;
        k_coef32<<<(unsigned)std::min<int64_t>((tot + 255) / 256, 65535), 256, 0, s>>>(base, c32, tot,
                                                                                      mom ? n : 0);
        CHNS_HIP(hipGetLastError());
        ok = true;
      }
      const float* cf[kMaxCoef] = {};
      for (int k = 0; k < nf; ++k) cf[k] = c32 + k * n;
      return mom ? apply_d<K_VP, float>(c, L, x, y, cf, s, o) : apply_d<K_CH_JAC, float>(c, L, x, y, cf, s, o);
    }
  }
  set_error("operator not available");
  return CHNS_EINVAL;
}

}  // namespace

int op_fields(int op, int dim) {
  switch (op) {
    case CHNS_OP_PRESSURE:
    case CHNS_OP_MASS:
    case CHNS_OP_MOMENTUM_SCALAR:
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

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept for the process.
int scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  CHNS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index beyond the library's limit");
    return CHNS_EINVAL;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    CHNS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = p;
  }
  *out = addr[dev];
  return CHNS_OK;
}

int launch_apply_noalloc(Ctx& c, int op, int prec, const void* x, void* y, hipStream_t s) {
  if (!c.scratch) {
    set_error("context has no scratch address");
    return CHNS_ESTATE;
  }
  const size_t es = prec == CHNS_FP64 ? sizeof(double) : sizeof(float);
  const int nf = op_fields(op, c.dm.dim);
  const size_t need = es * (size_t)nf * (size_t)(c.dm.n_slots > 0 ? c.dm.n_slots : 1);
  if (nf > 0 && need > kScratchBytes) {
    set_error("mesh needs " + std::to_string(need) + " bytes of slot scratch for this operator, more than the " +
              std::to_string(kScratchBytes) + " the allocation-free apply has");
    return CHNS_EINVAL;
  }
  LevelView L = fine_view(c);
  L.slots = c.scratch;
  ApplyOut o{};
  return launch_apply_lv(c, L, op, prec, x, y, s, o);
}

int launch_apply_lv(Ctx& c, const LevelView& L, int op, int prec, const void* x, void* y, hipStream_t s,
                    const ApplyOut& o) {
  if ((op == CHNS_OP_PRESSURE || op == CHNS_OP_MASS_RHO || op == CHNS_OP_MOMENTUM_SCALAR) && !c.phi_set) {
    set_error("set_phase_field must be called before this operator");
    return CHNS_ESTATE;
  }
  if ((op == CHNS_OP_MOMENTUM || op == CHNS_OP_CH_JACOBIAN) && L.dm != &c.dm) {
    set_error("the momentum and Cahn-Hilliard operators act on the fine mesh only");
    return CHNS_EINVAL;
  }
  if (prec == CHNS_FP64) return apply_dispatch<double>(c, L, op, (const double*)x, (double*)y, L.phi64, s, o);
  if (prec == CHNS_FP32) return apply_dispatch<float>(c, L, op, (const float*)x, (float*)y, L.phi32, s, o);
  set_error("prec must be CHNS_FP64 or CHNS_FP32");
  return CHNS_EINVAL;
}

int launch_apply(Ctx& c, int op, int prec, const void* x, void* y, hipStream_t s, const ApplyOut& o) {
  return launch_apply_lv(c, fine_view(c), op, prec, x, y, s, o);
}

static_assert((int)FORM_CH_RES == (int)K_CH_RES && (int)FORM_CH_JAC == (int)K_CH_JAC && (int)FORM_VP == (int)K_VP &&
                  (int)FORM_VP_RHS == (int)K_VP_RHS && (int)FORM_PP_RHS == (int)K_PP_RHS &&
                  (int)FORM_VU_RHS == (int)K_VU_RHS && (int)FORM_ENERGY == (int)K_ENERGY,
              "form numbering");

int launch_form(Ctx& c, int form, const double* x, const double* const* cf, double* y, hipStream_t s,
                const ApplyOut& o) {
  const LevelView L = fine_view(c);
  switch (form) {
    case FORM_CH_RES:
      return apply_d<K_CH_RES, double>(c, L, x, y, cf, s, o);
    case FORM_CH_JAC:
      return apply_d<K_CH_JAC, double>(c, L, x, y, cf, s, o);
    case FORM_VP:
      return apply_d<K_VP, double>(c, L, x, y, cf, s, o);
    case FORM_VP_RHS:
      return apply_d<K_VP_RHS, double>(c, L, x, y, cf, s, o);
    case FORM_PP_RHS:
      return apply_d<K_PP_RHS, double>(c, L, x, y, cf, s, o);
    case FORM_VU_RHS:
      return apply_d<K_VU_RHS, double>(c, L, x, y, cf, s, o);
    case FORM_ENERGY:
      return apply_d<K_ENERGY, double>(c, L, x, y, cf, s, o);
  }
  set_error("unknown form");
  return CHNS_EINVAL;
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
  // fields of the Cahn-Hilliard Jacobian are coupled: probe them one at a time
  const bool coupled = op == CHNS_OP_CH_JACOBIAN;
  for (int col = 0; col < L.dm->n_colors; ++col) {
    for (int f = coupled ? 0 : -1; f < (coupled ? nf : 0); ++f) {
      if (prec == CHNS_FP64)
        k_indicator<double><<<g, 256, 0, s>>>((double*)xi, L.dm->color, col, n, nf, f);
      else
        k_indicator<float><<<g, 256, 0, s>>>((float*)xi, L.dm->color, col, n, nf, f);
      CHNS_HIP(hipGetLastError());
      int rc = launch_apply_lv(c, L, op, prec, xi, yi, s, o);
      if (rc) return rc;
      if (prec == CHNS_FP64)
        k_take_diag<double><<<g, 256, 0, s>>>((double*)d, (const double*)yi, L.dm->color, col, n, nf, invert, f);
      else
        k_take_diag<float><<<g, 256, 0, s>>>((float*)d, (const float*)yi, L.dm->color, col, n, nf, invert, f);
      CHNS_HIP(hipGetLastError());
    }
  }
  return CHNS_OK;
}

// nf x nf node blocks of an FP64 operator (the couplings between the fields
// of one node), by probing every field of every colour class
int launch_block_diagonal(Ctx& c, int op, double* blk, double* xi, double* yi, hipStream_t s) {
  const LevelView L = fine_view(c);
  const int64_t n = L.dm->n;
  const int nf = op_fields(op, L.dm->dim);
  const unsigned g = (unsigned)((n + 255) / 256);
  ApplyOut o{};
  for (int col = 0; col < L.dm->n_colors; ++col)
    for (int f = 0; f < nf; ++f) {
      k_indicator<double><<<g, 256, 0, s>>>(xi, L.dm->color, col, n, nf, f);
      CHNS_HIP(hipGetLastError());
      int rc = launch_apply_lv(c, L, op, CHNS_FP64, xi, yi, s, o);
      if (rc) return rc;
      k_take_block<<<g, 256, 0, s>>>(blk, yi, L.dm->color, col, n, nf, f);
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
