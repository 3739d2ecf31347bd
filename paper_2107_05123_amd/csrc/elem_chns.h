// Element routines of the Cahn-Hilliard and VMS momentum forms (full 2-point
// Gauss quadrature per direction; FP64).  Each routine receives the corner
// values of its fields (corner a has coordinate bit d = (a >> d) & 1) and
// adds sum_q detJ (...) for every test function N_a.
//
// Paper: mixture laws and psi (Sec. 2), time averages (Sec. 3), discrete
// Cahn-Hilliard (Def. 6), VMS velocity prediction (Def. 3), tau_m and R_m
// (Sec. 3.1), VMS pressure Poisson (Def. 4), VMS velocity update (Def. 5).
// Readings: coefficients and nonlinear functions at the Gauss points;
// J = (rho- - rho+)/(2 rho+ Cn) grad mu~; G = (2/h)^2 I; inside R_m the Q1
// fields have no pure second derivatives, so the viscous part is
// grad eta~ . grad v and the capillary part sum_{j != i} d_i d_j phi~ d_j phi~.
#pragma once
#include <hip/hip_runtime.h>

namespace chns {

struct Phys {
  double dt, Pe, Cn, We, Re, Fr, C_I;
  double alpha, beta;  // rho(phi) = alpha phi* + beta
  double gam, xi;      // eta(phi) = gam phi* + xi
  double cJ;           // (rho- - rho+) / (2 rho+ Cn)
  int gaxis;
};

constexpr double kG = 0.57735026918962576451;

// reference Q1 tables on [-1,1]^d at the Gauss points (bit d of q / a)
template <int DIM>
__host__ __device__ constexpr double refN(int q, int a) {
  double v = 1.0;
  for (int d = 0; d < DIM; ++d) {
    const double sa = ((a >> d) & 1) ? 1.0 : -1.0, sq = ((q >> d) & 1) ? kG : -kG;
    v *= 0.5 * (1.0 + sa * sq);
  }
  return v;
}
template <int DIM>
__host__ __device__ constexpr double refD(int q, int a, int dd) {
  double v = 1.0;
  for (int d = 0; d < DIM; ++d) {
    const double sa = ((a >> d) & 1) ? 1.0 : -1.0, sq = ((q >> d) & 1) ? kG : -kG;
    v *= d == dd ? 0.5 * sa : 0.5 * (1.0 + sa * sq);
  }
  return v;
}
template <int DIM>
__host__ __device__ constexpr double refH(int q, int a, int i, int j) {
  double v = 1.0;
  for (int d = 0; d < DIM; ++d) {
    const double sa = ((a >> d) & 1) ? 1.0 : -1.0, sq = ((q >> d) & 1) ? kG : -kG;
    v *= (d == i || d == j) ? 0.5 * sa : 0.5 * (1.0 + sa * sq);
  }
  return v;
}

template <int DIM>
struct QP {
  static constexpr int NC = 1 << DIM;
  // value and physical gradient of a corner field at Gauss point q
  __device__ static inline double val(const double* f, int q) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < NC; ++a) s += refN<DIM>(q, a) * f[a];
    return s;
  }
  __device__ static inline void grad(const double* f, int q, double gs, double* g) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < NC; ++a) s += refD<DIM>(q, a, d) * f[a];
      g[d] = gs * s;
    }
  }
  __device__ static inline double hess(const double* f, int q, int i, int j, double gs2) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < NC; ++a) s += refH<DIM>(q, a, i, j) * f[a];
    return gs2 * s;
  }
};

__device__ inline double pull_back(double p) { return fmin(fmax(p, -1.0), 1.0); }
__device__ inline double dpsi(double p) { return p * p * p - p; }
__device__ inline double d2psi(double p) { return 3.0 * p * p - 1.0; }
__device__ inline double psi(double p) {
  const double t = p * p - 1.0;
  return 0.25 * t * t;
}

// Gauss-point quantities of the momentum forms.
template <int DIM>
struct MomQ {
  double rho, eta, tau, geta[DIM], uh[DIM], J[DIM], gphi[DIM], phi;
  __device__ inline void init(const Phys& P, const double* phit, const double* mut, const double* const* uhat, int q,
                              double gs) {
    phi = QP<DIM>::val(phit, q);
    const double ps = pull_back(phi);
    rho = P.alpha * ps + P.beta;
    eta = P.gam * ps + P.xi;
    QP<DIM>::grad(phit, q, gs, gphi);
    const double inside = fabs(phi) < 1.0 ? 1.0 : 0.0;
    double gm[DIM];
    QP<DIM>::grad(mut, q, gs, gm);
    double uu = 0.0, uJ = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      geta[d] = P.gam * gphi[d] * inside;
      uh[d] = QP<DIM>::val(uhat[d], q);
      J[d] = P.cJ * gm[d];
      uu += uh[d] * uh[d];
      uJ += uh[d] * J[d];
    }
    const double gs2 = gs * gs;
    const double r = eta / (rho * P.Re);
    const double arg = 4.0 / (P.dt * P.dt) + gs2 * uu + gs2 * uJ / (rho * P.Pe) + P.C_I * DIM * gs2 * gs2 * r * r;
    tau = 1.0 / sqrt(arg);
  }
  // stabilisation test function s_a = 1/2 u^.grad N_a + 1/(2 Pe rho) J.grad N_a
  __device__ inline double s(const Phys& P, const double* gNa) const {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      a += uh[d] * gNa[d];
      b += J[d] * gNa[d];
    }
    return 0.5 * a + b / (2.0 * P.Pe * rho);
  }
  // R_lin(v) from the value and gradient of v
  __device__ inline double rlin(const Phys& P, double v, const double* gv) const {
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      a += uh[d] * gv[d];
      b += J[d] * gv[d];
      c += geta[d] * gv[d];
    }
    return rho * v / P.dt + 0.5 * rho * a + b / (2.0 * P.Pe) - c / (2.0 * P.Re);
  }
  // known part of R_m for component i (u = u^k, p = p^k)
  __device__ inline double rknown(const Phys& P, int i, double ui, const double* gui, const double* gp,
                                  double kort) const {
    const double g = i == P.gaxis ? -1.0 : 0.0;
    return -rho * ui / P.dt + 0.5 * rho * dot(uh, gui) + dot(J, gui) / (2.0 * P.Pe) - dot(geta, gui) / (2.0 * P.Re) +
           P.Cn / P.We * kort + gp[i] - rho * g / P.Fr;
  }
  __device__ static inline double dot(const double* a, const double* b) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) s += a[d] * b[d];
    return s;
  }
};

// capillary divergence of R_m, component i
template <int DIM>
__device__ inline double kort_i(const double* phit, int q, int i, double gs, const double* gphi) {
  double k = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j)
    if (j != i) k += QP<DIM>::hess(phit, q, i, j, gs * gs) * gphi[j];
  return k;
}

template <int DIM>
__device__ inline void gradN(int q, int a, double gs, double* g) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) g[d] = gs * refD<DIM>(q, a, d);
}

}  // namespace chns
