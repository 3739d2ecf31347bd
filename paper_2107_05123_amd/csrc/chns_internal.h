// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>


#include "chns.h"
#include "mesh_host.h"

namespace chns {

void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define CHNS_HIP(call)                                  \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::chns::hip_fail(e_, #call); \
  } while (0)

// Device copy of one brick class.
struct DevBrickClass {
  int B = 0;
  int64_t count = 0;
  int npb = 0;            // nodes per brick
  int nbnd = 0;           // boundary positions per brick
  int64_t slot_base = 0;
  int32_t* table = nullptr;
  int8_t* level = nullptr;
  int16_t* rank = nullptr;  // npb entries
  int32_t* anchor = nullptr;  // 3 per brick (integer node coordinates)
  int32_t* abase = nullptr;   // 8 per brick, or null (see BrickClass::abase)
};

struct DevMesh {
  int dim = 3;
  int max_level = 0;
  int64_t n = 0;           // independent nodes
  int64_t n_hanging = 0;
  int64_t n_slots = 0;
  DevBrickClass cls[kBrickClasses];
  int32_t* hang_par = nullptr;  // n_hanging * 4, -1 padded
  int64_t n_comb = 0;
  int32_t* comb_node = nullptr;
  int32_t* comb_ptr = nullptr;
  uint32_t* comb_ent = nullptr;
  uint8_t* color = nullptr;
  uint8_t* wall = nullptr;
  int n_colors = 0;
  bool structured = false;  // uniform mesh, lexicographic node numbers
  int32_t side = 0;         // 2^max_level
};

// Scalars of one Krylov solve kept on the device.
struct DevScalars {
  double pq, rz, rz_old, rr, bb, alpha, beta, sum;
  double tol2;        // (rtol |b|)^2
  int it, done, max_it;
  int phi_bad;  // set by chns_set_phase_field when phi~ holds a NaN or an infinity
};

// One coarse level of the geometric multigrid hierarchy (level 0 is the
// context's own mesh and fields).
struct MgLevel {
  HostMesh host;
  DevMesh dm;
  double* phi64 = nullptr;
  float* phi32 = nullptr;
  void* slots = nullptr;
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  double* v64[4] = {};  // rhs, solution, temporary, probe output
  float* v32[4] = {};
  // rows on the next finer level: prolongation from this level
  int64_t P_rows = 0;
  int32_t *P_ptr = nullptr, *P_col = nullptr;
  double* P_val64 = nullptr;
  float* P_val32 = nullptr;
  // rows on this level: restriction (P^T) and injection of nodal fields
  int32_t *R_ptr = nullptr, *R_col = nullptr;
  double* R_val64 = nullptr;
  float* R_val32 = nullptr;
  int32_t *I_ptr = nullptr, *I_col = nullptr;
  double* I_val = nullptr;
  // structured levels above the coarsest: the assembled operator as a
  // (3^d)-point stencil, SoA [offset][node], offsets x fastest over -1..1
  double* S64 = nullptr;
  float* S32 = nullptr;
  double* E64 = nullptr;  // element matrices of those levels (NC^2 per leaf)
  // coarsest level: dense inverse of the rank-one regularised operator
  double* inv64 = nullptr;
  float* inv32 = nullptr;
  double* dense = nullptr;
};

struct Multigrid {
  std::vector<MgLevel> lv;  // lv[0] unused placeholder for the fine level
  double* fine_dinv64 = nullptr;
  float* fine_dinv32 = nullptr;
  double* fine_t64 = nullptr;
  float* fine_t32 = nullptr;
  // reference tables of the element-matrix Galerkin products (device):
  // G (q, a, b), P (c, b, A), H (c, q, A, B); H only when the fine level is
  // uniform and feeds the first coarse level directly
  double* tab_G = nullptr;
  double* tab_P = nullptr;
  double* tab_H = nullptr;
  double* tab_M = nullptr;  // reference mass sum_q N_a N_b (for a mass shift)
  // per-Gauss-point reference mass Mq (q, a, b) and its Galerkin products
  // Hm (c, q, A, B) = P_c^T Mq_q P_c (variable-density mass)
  double* tab_Mq = nullptr;
  double* tab_Hm = nullptr;
  double* diag_part = nullptr;  // 3^d fine-diagonal partials per first-coarse-level element
  bool setup_valid = false;
  hipGraphExec_t setup_exec = nullptr;  // captured device part of the set-up
  hipGraphExec_t mom_setup_exec = nullptr;  // the same for the scalar momentum operator
  // captured set-ups of shifted operators (mass shift, graph)
  std::vector<std::pair<double, hipGraphExec_t>> shifted_setups;
  bool transfer32_exact = false;  // every transfer weight is exact in FP32
  int nu = 2;            // damped-Jacobi sweeps before and after the correction (per set-up)
  double omega = 0.6;    // damping (per set-up)
};

struct Ctx {
  chns_mesh* mesh_handle = nullptr;
  const HostMesh* host = nullptr;
  DevMesh dm;
  chns_params prm{};
  int device = 0;
  std::vector<void*> allocs;

  // phase field phi~ in both precisions
  double* phi64 = nullptr;
  float* phi32 = nullptr;
  bool phi_set = false;

  // slot buffers (largest field count * n_slots), both precisions share storage
  void* slots = nullptr;
  size_t slots_bytes = 0;
  // device address of the per-GPU slot scratch of the allocation-free apply
  void* scratch = nullptr;

  // reduction scratch
  double* partials = nullptr;   // kMaxPartials
  unsigned* counter = nullptr;  // ticket counters
  DevScalars* sc = nullptr;     // device scalars
  DevScalars* sc_host = nullptr;  // pinned mirror
  // pinned host words {done, it} that the CG finaliser stores to directly
  // (system scope), so convergence polling needs no copy on the stream
  int* flag_host = nullptr;

  // work vectors (lazily allocated)
  double* w64[8] = {};
  float* w32[8] = {};
  double* diag64 = nullptr;  // inverse diagonal of the pressure operator
  float* diag32 = nullptr;
  bool diag_valid = false;

  Multigrid* mg = nullptr;
  // mass shift g of the pressure operator (K_{1/rho} + g M): 0 for the
  // public operator; set only while the Cahn-Hilliard preconditioner uses
  // the multigrid hierarchy
  double pp_shift = 0.0;
  // 1: the "pressure" operator stands for the scalar momentum operator
  // K_{eta(phi)/(2 Re)} + M_{rho(phi)/dt} (one velocity component) while the
  // velocity-prediction preconditioner uses the multigrid hierarchy; 0 otherwise
  int pp_kind = 0;

  // coefficient fields of the momentum and Cahn-Hilliard Jacobian operators
  // (context-owned copies, (2 + dim) * n each): [phi~, mu~, u^] and
  // [phi^{k+1}, phi^k, u~]
  double* coef_mom = nullptr;
  double* coef_chj = nullptr;
  bool coef_mom_set = false, coef_chj_set = false;
  // FP32 copies for the FP32 applies (momentum phase field as 1 + phi~),
  // refreshed lazily after the FP64 fields change
  float* coef_mom32 = nullptr;
  float* coef_chj32 = nullptr;
  bool coef_mom32_ok = false, coef_chj32_ok = false;

  struct Stepper* step = nullptr;  // time-step work arrays (chns_step.hip)
  struct UNet* unet = nullptr;     // learned preconditioner (unet.hip)

  // solves run on a context-owned stream (default priority) so that their
  // iterations can be captured into HIP graphs, cached per configuration
  hipStream_t work = nullptr;
  hipEvent_t ev_in = nullptr;
  struct GraphEntry {
    int prec, pc, flexible, op;
    const void* x;
    const void* dinv;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  double* xw64 = nullptr;  // solution buffer of FP64 solves (fixed address for graphs)
  hipGraphExec_t diag_exec = nullptr;  // captured Jacobi diagonal set-up

  // optional per-kernel HIP-event timers (tagged launch groups)
  bool prof = false;
  struct ProfRec {
    std::string tag;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  struct ProfAcc {
    std::string tag;
    double ms;
    int64_t launches;
  };
  std::vector<ProfAcc> prof_acc;
  hipEvent_t prof_event();
  void prof_begin(const char* tag, hipStream_t s, hipEvent_t* start);
  void prof_end(const char* tag, hipStream_t s, hipEvent_t start);

  void* dalloc(size_t bytes);
  ~Ctx();
};

// slot scratch of the allocation-free apply, per GPU (apply.hip)
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
constexpr int kMaxPartials = 1 << 20;  // per-block reduction partials (bricks + combine blocks of the largest meshes)
constexpr int kMaxCoefFields = 16;  // coefficient fields one element form may read

// A mesh level as seen by the apply kernels: the fine level of a context or
// one level of its multigrid hierarchy.
struct LevelView {
  const DevMesh* dm;
  const double* phi64;
  const float* phi32;
  void* slots;
};

// ---- apply (apply.hip)
struct ApplyOut {
  // optional fused reduction: sum_i x_i * y_i over written nodes into sc->pq
  bool fuse_dot = false;
  const int* done = nullptr;  // skip all work when *done != 0
  // pressure operator only: a damped-Jacobi sweep instead of the product,
  // y = x + w dinv (r - A x) (y must not alias x); vectors of the apply's
  // precision
  const void* sm_r = nullptr;
  const void* sm_dinv = nullptr;
  double sm_w = 0.0;
};
int launch_apply(Ctx& c, int op, int prec, const void* x, void* y, hipStream_t s, const ApplyOut& o);
int launch_apply_lv(Ctx& c, const LevelView& L, int op, int prec, const void* x, void* y, hipStream_t s,
                    const ApplyOut& o);
int launch_diagonal(Ctx& c, int op, int prec, void* dinv_or_d, bool invert, hipStream_t s);
// probing with caller-provided work vectors xi, yi (n * fields each)
int launch_diagonal_lv(Ctx& c, const LevelView& L, int op, int prec, void* d, bool invert, void* xi, void* yi,
                       hipStream_t s);
LevelView fine_view(Ctx& c);
int op_fields(int op, int dim);
// device copy of a host mesh (brick tables, combine rows, colours, walls)
int upload_dm(Ctx& c, const HostMesh& m, DevMesh& d);
// address of the per-GPU static slot scratch on the current device (looked
// up once per device); the apply below uses it instead of the context's slots
int scratch_address(void** out);
int launch_apply_noalloc(Ctx& c, int op, int prec, const void* x, void* y, hipStream_t s);

// Run `enqueue(stream)` through a HIP graph captured on first use and cached
// in *cache (eagerly when profiling).  The enqueued work must be kernels only.
template <class F>
int run_captured(Ctx& c, hipGraphExec_t* cache, hipStream_t s, F&& enqueue) {
  if (c.prof) return enqueue(s);
  if (!*cache) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int rc = enqueue(s);
    e = hipStreamEndCapture(s, &g);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(cache, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  }
  hipError_t e = hipGraphLaunch(*cache, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return CHNS_OK;
}

// Element forms beyond the public operators (numbering shared with the
// apply kernels).  Fields (each n long, vectors component-blocked):
//   CH_RES  x = [phi^{k+1}, mu^{k+1}], cf = [phi^k, mu^k, u~_0..]    -> 2 fields
//   CH_JAC  x = [dphi, dmu],           cf = [phi^{k+1}, phi^k, u~]   -> 2 fields
//   VP      x = v (dim),               cf = [phi~, mu~, u^]          -> dim fields
//   VP_RHS  cf = [phi~, mu~, u^, u^k, p^k, f_v]                     -> dim fields
//   PP_RHS  cf = [phi~, mu~, u^, u^k, p^k, v, f_v]                  -> 1 field
//   VU_RHS  cf = [phi~, mu~, u^, u^k, p^k, v, p^{k+1}, f_v]         -> dim fields
//   (f_v: body force of the momentum equation, dim fields; zeros without one)
//   ENERGY  cf = [phi, vertical coordinate, u]                       -> 1 field
enum Form { FORM_CH_RES = 3, FORM_CH_JAC = 4, FORM_VP = 5, FORM_VP_RHS = 6, FORM_PP_RHS = 7, FORM_VU_RHS = 8,
            FORM_ENERGY = 9 };
int launch_form(Ctx& c, int form, const double* x, const double* const* cf, double* y, hipStream_t s,
                const ApplyOut& o);
int launch_block_diagonal(Ctx& c, int op, double* blk, double* xi, double* yi, hipStream_t s);

// ---- geometric multigrid (gmg.hip)
int mg_build(Ctx& c);
int mg_setup(Ctx& c, hipStream_t s);
int mg_vcycle64(Ctx& c, const double* r, double* z, hipStream_t s);
// y = P x per field (CSR P: rows x cols; x, y field-blocked, nf fields)
int interp_apply(const int32_t* ptr, const int32_t* col, const double* val, int64_t rows, int64_t cols, int nf,
                 const double* x, double* y, hipStream_t s);
int mg_vcycle32(Ctx& c, const float* r, float* z, hipStream_t s);

// ---- krylov (krylov.hip)
int launch_set_phase(Ctx& c, const double* phi, const double* prev, hipStream_t s);
int solve_pressure_impl(Ctx& c, const double* b, double* x, const chns_solve_opts& o, chns_solve_stats& st,
                        hipStream_t s);
// Jacobi-preconditioned CG to |b - A x| <= rtol |b| for an SPD operator (no
// projection), on the calling stream; x in/out (n_fields * n).
int solve_spd_impl(Ctx& c, int op, const double* b, double* x, const double* dinv, double rtol, int max_it,
                   bool graphs, hipStream_t s, int* iters, double* rel);

// ---- learned preconditioner (unet.hip)
int unet_create(Ctx& c);
void unet_destroy(Ctx& c);
int unet_init(Ctx& c, uint64_t seed, float K, float omega, hipStream_t s);
int unet_load(Ctx& c, const void* blob, size_t n, hipStream_t s);
int unet_save(Ctx& c, void* blob, size_t cap, size_t* n);
int unet_gradients(Ctx& c, float* host, size_t n);
size_t unet_param_count(const Ctx& c);
int unet_forward_crop(Ctx& c, const double* phi, const double* r, const int32_t* origin, int flip, int crop,
                      float* out, hipStream_t s);
int unet_train_step(Ctx& c, const chns_pc_batch& b, float lr, float* loss, hipStream_t s);
int unet_prepare(Ctx& c, hipStream_t s);
bool unet_ready(const Ctx& c);
template <typename T>
int unet_apply(Ctx& c, const T* r, T* z, hipStream_t s);

// ---- CHNS time step (chns_step.hip)
int set_coefficients_impl(Ctx& c, int op, const double* const* fields, hipStream_t s);
int assemble_impl(Ctx& c, int form, const double* const* fields, double* out, hipStream_t s);
int initial_mu_impl(Ctx& c, const double* phi, double* mu, hipStream_t s);
int advance_step_impl(Ctx& c, const chns_state& st, const chns_step_opts& o, chns_step_stats& stats,
                      hipStream_t s);
void destroy_stepper(Ctx& c);

}  // namespace chns

struct chns_mesh {
  chns::HostMesh m;
};
struct chns_transfer {
  int64_t rows = 0, cols = 0;
  std::vector<int32_t> ptr, col;
  std::vector<double> val;
  // device copy, uploaded by the first apply
  int device = -1;
  int32_t *d_ptr = nullptr, *d_col = nullptr;
  double* d_val = nullptr;
  ~chns_transfer();
};
struct chns_ctx {
  chns::Ctx c;
};
