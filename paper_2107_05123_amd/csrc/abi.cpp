// C ABI entry points of libchns (declared in include/chns.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "chns_internal.h"

namespace chns {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return CHNS_EHIP;
}

void* Ctx::dalloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    set_error("hipMalloc failed (" + std::to_string(bytes) + " bytes)");
    return nullptr;
  }
  allocs.push_back(p);
  return p;
}

hipEvent_t Ctx::prof_event() {
  if (!prof_pool.empty()) {
    hipEvent_t e = prof_pool.back();
    prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Ctx::prof_begin(const char* tag, hipStream_t s, hipEvent_t* start) {
  *start = nullptr;
  if (!prof) return;
  *start = prof_event();
  if (*start) (void)hipEventRecord(*start, s);
}

void Ctx::prof_end(const char* tag, hipStream_t s, hipEvent_t start) {
  if (!prof || !start) return;
  hipEvent_t stop = prof_event();
  if (!stop) return;
  (void)hipEventRecord(stop, s);
  prof_pending.push_back({tag, start, stop});
}

Ctx::~Ctx() {
  destroy_stepper(*this);
  unet_destroy(*this);
  if (mg && mg->setup_exec) (void)hipGraphExecDestroy(mg->setup_exec);
  if (mg && mg->mom_setup_exec) (void)hipGraphExecDestroy(mg->mom_setup_exec);
  if (mg)
    for (auto& e : mg->shifted_setups)
      if (e.second) (void)hipGraphExecDestroy(e.second);
  if (diag_exec) (void)hipGraphExecDestroy(diag_exec);
  delete mg;
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
  if (ev_in) (void)hipEventDestroy(ev_in);
  if (work) (void)hipStreamDestroy(work);
  for (auto& r : prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : prof_pool) (void)hipEventDestroy(e);
  for (void* p : allocs) (void)hipFree(p);
  if (sc_host) (void)hipHostFree(sc_host);
  if (flag_host) (void)hipHostFree(flag_host);
}

}  // namespace chns

using namespace chns;

#define CHNS_GUARD_BEGIN try {
#define CHNS_GUARD_END                                  \
  }                                                     \
  catch (const std::bad_alloc&) {                       \
    set_error("host allocation failed");                \
    return CHNS_ENOMEM;                                 \
  }                                                     \
  catch (...) {                                         \
    set_error("unexpected internal exception");         \
    return CHNS_EINVAL;                                 \
  }

extern "C" {

const char* chns_last_error(void) { return g_err.c_str(); }
const char* chns_version(void) { return "libchns 0.1 (gfx950)"; }

int chns_octree_build(const chns_mesh_spec* spec, chns_mesh** out) {
  CHNS_GUARD_BEGIN
  if (!spec || !out) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  *out = nullptr;
  auto* m = new chns_mesh();
  std::string msg;
  int rc = build_host_mesh(*spec, m->m, msg);
  if (rc) {
    set_error(msg);
    delete m;
    return rc;
  }
  *out = m;
  return CHNS_OK;
  CHNS_GUARD_END
}

int chns_mesh_destroy(chns_mesh* mesh) {
  delete mesh;
  return CHNS_OK;
}

int chns_mesh_info_get(const chns_mesh* mesh, chns_mesh_info* out) {
  if (!mesh || !out) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  const HostMesh& m = mesh->m;
  std::memset(out, 0, sizeof(*out));
  out->dim = m.dim;
  out->max_level = m.max_level;
  out->node_order = m.node_order;
  out->uniform = m.uniform ? 1 : 0;
  out->n_elems = m.n_elems();
  out->n_nodes = m.n_indep;
  out->n_hanging = m.n_hanging;
  for (int k = 0; k < kBrickClasses; ++k) {
    out->n_bricks[k] = m.cls[k].count;
    int64_t per = 1;
    for (int d = 0; d < m.dim; ++d) per *= m.cls[k].B;
    out->elems_in_bricks[k] = m.cls[k].count * per;
  }
  out->n_slots = m.n_slots;
  out->n_shared = (int64_t)m.comb_node.size();
  out->n_colors = m.n_colors;
  for (auto l : m.leaf_level)
    if (l >= 0 && l <= 16) out->level_counts[(int)l]++;
  for (int d = 0; d < 3; ++d) out->box[d] = m.box_hi[d];
  return CHNS_OK;
}

int chns_mesh_node_coords(const chns_mesh* mesh, int64_t* ijk) {
  if (!mesh || !ijk) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  const HostMesh& m = mesh->m;
  for (int64_t i = 0; i < m.n_indep; ++i)
    for (int d = 0; d < m.dim; ++d) ijk[i * m.dim + d] = m.indep_coords[3 * i + d];
  return CHNS_OK;
}

int chns_mesh_leaves(const chns_mesh* mesh, int32_t* level, int64_t* anchor) {
  if (!mesh || !level || !anchor) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  const HostMesh& m = mesh->m;
  for (int64_t e = 0; e < m.n_elems(); ++e) {
    level[e] = m.leaf_level[e];
    for (int d = 0; d < m.dim; ++d) anchor[e * m.dim + d] = m.leaf_anchor[3 * e + d];
  }
  return CHNS_OK;
}

int chns_mesh_hanging(const chns_mesh* mesh, int64_t* coords, int32_t* parents) {
  if (!mesh || !coords || !parents) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  const HostMesh& m = mesh->m;
  for (int64_t h = 0; h < m.n_hanging; ++h) {
    for (int d = 0; d < m.dim; ++d) coords[h * m.dim + d] = m.hang_coords[3 * h + d];
    for (int q = 0; q < 4; ++q) parents[4 * h + q] = m.hang_parents[4 * h + q];
  }
  return CHNS_OK;
}

int chns_mesh_remesh(const chns_mesh* old, const double* phi, int min_level, double threshold, int brick_max,
                     chns_mesh** out) {
  CHNS_GUARD_BEGIN
  if (!old || !phi || !out) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  *out = nullptr;
  auto* m = new chns_mesh();
  std::string msg;
  int rc = build_host_mesh_remesh(old->m, phi, min_level, threshold, brick_max, m->m, msg);
  if (rc) {
    set_error(msg);
    delete m;
    return rc;
  }
  *out = m;
  return CHNS_OK;
  CHNS_GUARD_END
}

chns_transfer::~chns_transfer() {
  if (d_ptr) (void)hipFree(d_ptr);
  if (d_col) (void)hipFree(d_col);
  if (d_val) (void)hipFree(d_val);
}

int chns_transfer_create(const chns_mesh* from, const chns_mesh* to, chns_transfer** out) {
  CHNS_GUARD_BEGIN
  if (!from || !to || !out) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  *out = nullptr;
  auto* t = new chns_transfer();
  std::string msg;
  int rc = build_interp(from->m, to->m, t->ptr, t->col, t->val, msg);
  if (rc) {
    set_error(msg);
    delete t;
    return rc;
  }
  t->rows = to->m.n_indep;
  t->cols = from->m.n_indep;
  *out = t;
  return CHNS_OK;
  CHNS_GUARD_END
}

int chns_transfer_info(const chns_transfer* t, int64_t* rows, int64_t* cols, int64_t* nnz) {
  if (!t || !rows || !cols || !nnz) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  *rows = t->rows;
  *cols = t->cols;
  *nnz = (int64_t)t->val.size();
  return CHNS_OK;
}

int chns_transfer_matrix(const chns_transfer* t, int32_t* ptr, int32_t* col, double* val) {
  if (!t || !ptr || (!t->val.empty() && (!col || !val))) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  std::copy(t->ptr.begin(), t->ptr.end(), ptr);
  std::copy(t->col.begin(), t->col.end(), col);
  std::copy(t->val.begin(), t->val.end(), val);
  return CHNS_OK;
}

int chns_transfer_apply(chns_transfer* t, int n_fields, const double* x, double* y, void* stream) {
  CHNS_GUARD_BEGIN
  if (!t || !x || !y || n_fields < 1 || (const void*)x == (const void*)y) {
    set_error("null argument, n_fields < 1 or aliased x and y");
    return CHNS_EINVAL;
  }
  int dev = 0;
  CHNS_HIP(hipGetDevice(&dev));
  if (t->device != dev) {
    if (t->device >= 0) {
      set_error("transfer was uploaded to another device");
      return CHNS_EINVAL;
    }
    const size_t nnz = t->val.size();
    int32_t *dp = nullptr, *dc = nullptr;
    double* dv = nullptr;
    hipError_t e = hipMalloc(&dp, sizeof(int32_t) * t->ptr.size());
    if (e == hipSuccess) e = hipMalloc(&dc, sizeof(int32_t) * std::max<size_t>(nnz, 1));
    if (e == hipSuccess) e = hipMalloc(&dv, sizeof(double) * std::max<size_t>(nnz, 1));
    if (e == hipSuccess) e = hipMemcpy(dp, t->ptr.data(), sizeof(int32_t) * t->ptr.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz) e = hipMemcpy(dc, t->col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz) e = hipMemcpy(dv, t->val.data(), sizeof(double) * nnz, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      // nothing kept: a later call can try again
      if (dp) (void)hipFree(dp);
      if (dc) (void)hipFree(dc);
      if (dv) (void)hipFree(dv);
      return hip_fail(e, "transfer upload");
    }
    t->d_ptr = dp;
    t->d_col = dc;
    t->d_val = dv;
    t->device = dev;
  }
  return interp_apply(t->d_ptr, t->d_col, t->d_val, t->rows, t->cols, n_fields, x, y, (hipStream_t)stream);
  CHNS_GUARD_END
}

int chns_transfer_destroy(chns_transfer* t) {
  delete t;
  return CHNS_OK;
}

int chns_context_create(chns_mesh* mesh, const chns_params* params, chns_ctx** out) {
  CHNS_GUARD_BEGIN
  if (!mesh || !params || !out) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  *out = nullptr;
  if (!(params->rho_plus > 0.0) || !(params->rho_minus > 0.0)) {
    set_error("densities must be positive");
    return CHNS_EINVAL;
  }
  auto* h = new chns_ctx();
  Ctx& c = h->c;
  c.mesh_handle = mesh;
  c.host = &mesh->m;
  c.prm = *params;
  if (c.prm.Pe <= 0.0) c.prm.Pe = 1.0 / (3.0 * c.prm.Cn * c.prm.Cn);
  if (c.prm.C_I <= 0.0) c.prm.C_I = 6.0;
  int rc = CHNS_OK;
  if (hipGetDevice(&c.device) != hipSuccess) {
    set_error("no HIP device available");
    delete h;
    return CHNS_EHIP;
  }
  rc = upload_dm(c, *c.host, c.dm);
  const int64_t n = c.dm.n;
  if (!rc) {
    c.phi64 = (double*)c.dalloc(sizeof(double) * n);
    c.phi32 = (float*)c.dalloc(sizeof(float) * n);
    c.slots_bytes = sizeof(double) * (size_t)(c.dm.n_slots > 0 ? c.dm.n_slots : 1) * 3;
    c.slots = c.dalloc(c.slots_bytes);
    c.partials = (double*)c.dalloc(sizeof(double) * kMaxPartials);
    c.counter = (unsigned*)c.dalloc(sizeof(unsigned) * 16);
    c.sc = (DevScalars*)c.dalloc(sizeof(DevScalars));
    if (!c.phi64 || !c.phi32 || !c.slots || !c.partials || !c.counter || !c.sc) rc = CHNS_ENOMEM;
  }
  if (!rc && hipMemset(c.counter, 0, sizeof(unsigned) * 16) != hipSuccess) rc = hip_fail(hipErrorUnknown, "memset");
  if (!rc && hipMemset(c.sc, 0, sizeof(DevScalars)) != hipSuccess) rc = hip_fail(hipErrorUnknown, "memset");
  if (!rc && hipHostMalloc((void**)&c.sc_host, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess)
    rc = hip_fail(hipErrorOutOfMemory, "hipHostMalloc");
  if (!rc && hipHostMalloc((void**)&c.flag_host, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    rc = hip_fail(hipErrorOutOfMemory, "hipHostMalloc");
  if (!rc) c.flag_host[0] = c.flag_host[1] = 0;
  if (!rc && hipStreamCreateWithFlags(&c.work, hipStreamNonBlocking) != hipSuccess)
    rc = hip_fail(hipErrorUnknown, "hipStreamCreateWithFlags");
  if (!rc && hipEventCreateWithFlags(&c.ev_in, hipEventDisableTiming) != hipSuccess)
    rc = hip_fail(hipErrorUnknown, "hipEventCreateWithFlags");
  if (!rc) rc = scratch_address(&c.scratch);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return CHNS_OK;
  CHNS_GUARD_END
}

int chns_context_destroy(chns_ctx* ctx) {
  if (ctx) {
    (void)hipDeviceSynchronize();
    delete ctx;
  }
  return CHNS_OK;
}

int chns_set_phase_field(chns_ctx* ctx, const double* phi, const double* phi_prev, void* stream) {
  if (!ctx || !phi) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  return launch_set_phase(ctx->c, phi, phi_prev, (hipStream_t)stream);
}

int chns_apply_operator(chns_ctx* ctx, int op, int prec, const void* x, void* y, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !x || !y) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  if (x == y) {
    set_error("x and y must not alias");
    return CHNS_EINVAL;
  }
  ApplyOut o{};
  return launch_apply(ctx->c, op, prec, x, y, (hipStream_t)stream, o);
  CHNS_GUARD_END
}

int chns_apply_operator_noalloc(chns_ctx* ctx, int op, int prec, const void* x, void* y, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !x || !y) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  if (x == y) {
    set_error("x and y must not alias");
    return CHNS_EINVAL;
  }
  if (ctx->c.prof) {
    set_error("the allocation-free apply does not run with profiling enabled");
    return CHNS_EINVAL;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != ctx->c.device) {
    set_error("the current device is not the context's device");
    return CHNS_EINVAL;
  }
  return launch_apply_noalloc(ctx->c, op, prec, x, y, (hipStream_t)stream);
  CHNS_GUARD_END
}

int chns_operator_diagonal(chns_ctx* ctx, int op, int prec, void* d, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !d) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  return launch_diagonal(ctx->c, op, prec, d, false, (hipStream_t)stream);
  CHNS_GUARD_END
}

int chns_solve_pressure(chns_ctx* ctx, const double* b, double* x, const chns_solve_opts* opts,
                        chns_solve_stats* stats, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !b || !x) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  chns_solve_opts o{};
  o.rtol = 1e-8;
  o.max_it = 20000;
  o.pc = CHNS_PC_JACOBI;
  o.mode = CHNS_MODE_FP64;
  o.inner_rtol = 1e-4;
  o.check_every = 16;
  o.max_outer = 30;
  o.no_graphs = 0;
  if (opts) {
    o = *opts;
    if (!(o.rtol > 0.0)) o.rtol = 1e-8;
    if (o.max_it <= 0) o.max_it = 20000;
    if (!(o.inner_rtol > 0.0)) o.inner_rtol = 1e-4;
    if (o.check_every <= 0) o.check_every = 16;
    if (o.max_outer <= 0) o.max_outer = 30;
  }
  chns_solve_stats st{};
  int rc = solve_pressure_impl(ctx->c, b, x, o, st, (hipStream_t)stream);
  if (stats) *stats = st;
  return rc;
  CHNS_GUARD_END
}

int chns_set_coefficients(chns_ctx* ctx, int op, const double* const* fields, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  return set_coefficients_impl(ctx->c, op, fields, (hipStream_t)stream);
  CHNS_GUARD_END
}

int chns_assemble(chns_ctx* ctx, int form, const double* const* fields, double* out, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  return assemble_impl(ctx->c, form, fields, out, (hipStream_t)stream);
  CHNS_GUARD_END
}

int chns_initial_mu(chns_ctx* ctx, const double* phi, double* mu, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !phi || !mu) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  Ctx& c = ctx->c;
  CHNS_HIP(hipEventRecord(c.ev_in, (hipStream_t)stream));
  CHNS_HIP(hipStreamWaitEvent(c.work, c.ev_in, 0));
  int rc = initial_mu_impl(c, phi, mu, c.work);
  if (rc) return rc;
  CHNS_HIP(hipStreamSynchronize(c.work));
  return CHNS_OK;
  CHNS_GUARD_END
}

int chns_advance_step(chns_ctx* ctx, chns_state* state, const chns_step_opts* opts, chns_step_stats* stats,
                      void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !state || !state->u || !state->u_prev || !state->p || !state->phi || !state->mu) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  chns_step_opts o{};
  o.blocks = 2;
  o.newton_rtol = 1e-8;
  o.newton_atol = 1e-12;
  o.max_newton = 20;
  o.lin_rtol = 1e-8;
  o.max_it = 5000;
  o.restart = 64;
  o.pp_pc = CHNS_PC_JACOBI;
  o.pp_mode = CHNS_MODE_FP64;
  o.no_graphs = 0;
  if (opts) {
    o = *opts;
    if (o.blocks <= 0) o.blocks = 2;
    if (!(o.newton_rtol > 0.0)) o.newton_rtol = 1e-8;
    if (!(o.newton_atol > 0.0)) o.newton_atol = 1e-12;
    if (o.max_newton <= 0) o.max_newton = 20;
    if (!(o.lin_rtol > 0.0)) o.lin_rtol = 1e-8;
    if (o.max_it <= 0) o.max_it = 5000;
    if (o.restart <= 0) o.restart = 64;
  }
  if (o.ch_pc != CHNS_CH_PC_BLOCK_JACOBI && o.ch_pc != CHNS_CH_PC_SCHUR_GMG) {
    set_error("unknown Cahn-Hilliard preconditioner");
    return CHNS_EINVAL;
  }
  if (o.vp_pc != CHNS_VP_PC_JACOBI && o.vp_pc != CHNS_VP_PC_GMG) {
    set_error("unknown velocity-prediction preconditioner");
    return CHNS_EINVAL;
  }
  chns_step_stats st{};
  int rc = advance_step_impl(ctx->c, *state, o, st, (hipStream_t)stream);
  if (stats) *stats = st;
  return rc;
  CHNS_GUARD_END
}

int chns_pc_init(chns_ctx* ctx, uint64_t seed, float out_scale, float smooth_omega, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !(out_scale >= 0.0f) || !(smooth_omega >= 0.0f && smooth_omega < 2.0f)) {
    set_error("null context, negative output scale or damping outside [0, 2)");
    return CHNS_EINVAL;
  }
  return unet_init(ctx->c, seed, out_scale, smooth_omega, (hipStream_t)stream);
  CHNS_GUARD_END
}

int chns_pc_load(chns_ctx* ctx, const void* blob, size_t n, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !blob) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  return unet_load(ctx->c, blob, n, (hipStream_t)stream);
  CHNS_GUARD_END
}

int chns_pc_save(chns_ctx* ctx, void* blob, size_t cap, size_t* n) {
  CHNS_GUARD_BEGIN
  if (!ctx || !n) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  return unet_save(ctx->c, blob, cap, n);
  CHNS_GUARD_END
}

int chns_pc_param_count(chns_ctx* ctx, size_t* n) {
  CHNS_GUARD_BEGIN
  if (!ctx || !n) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  int rc = unet_create(ctx->c);
  if (rc) return rc;
  *n = unet_param_count(ctx->c);
  return CHNS_OK;
  CHNS_GUARD_END
}

int chns_pc_gradients(chns_ctx* ctx, float* host, size_t n) {
  CHNS_GUARD_BEGIN
  if (!ctx || !host) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  return unet_gradients(ctx->c, host, n);
  CHNS_GUARD_END
}

int chns_pc_forward(chns_ctx* ctx, const double* phi, const double* r, const int32_t* origin, int flip, int crop,
                    float* out, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !phi || !r || !origin || !out) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  return unet_forward_crop(ctx->c, phi, r, origin, flip, crop, out, (hipStream_t)stream);
  CHNS_GUARD_END
}

int chns_pc_train_step(chns_ctx* ctx, const chns_pc_batch* batch, float lr, float* loss, void* stream) {
  CHNS_GUARD_BEGIN
  if (!ctx || !batch) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  return unet_train_step(ctx->c, *batch, lr, loss, (hipStream_t)stream);
  CHNS_GUARD_END
}

int chns_profile_enable(chns_ctx* ctx, int enable) {
  if (!ctx) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  ctx->c.prof = enable != 0;
  return CHNS_OK;
}

int chns_profile_read(chns_ctx* ctx, const char* tag, double* ms, int64_t* launches) {
  if (!ctx || !tag || !ms || !launches) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  Ctx& c = ctx->c;
  for (auto& r : c.prof_pending) {
    CHNS_HIP(hipEventSynchronize(r.b));
    float t = 0.0f;
    CHNS_HIP(hipEventElapsedTime(&t, r.a, r.b));
    bool found = false;
    for (auto& acc : c.prof_acc)
      if (acc.tag == r.tag) {
        acc.ms += t;
        acc.launches += 1;
        found = true;
      }
    if (!found) c.prof_acc.push_back({r.tag, (double)t, 1});
    c.prof_pool.push_back(r.a);
    c.prof_pool.push_back(r.b);
  }
  c.prof_pending.clear();
  *ms = 0.0;
  *launches = 0;
  for (auto& acc : c.prof_acc)
    if (acc.tag == tag) {
      *ms = acc.ms;
      *launches = acc.launches;
    }
  return CHNS_OK;
}

int chns_profile_reset(chns_ctx* ctx) {
  if (!ctx) {
    set_error("null argument");
    return CHNS_EINVAL;
  }
  double ms;
  int64_t n;
  chns_profile_read(ctx, "", &ms, &n);
  ctx->c.prof_acc.clear();
  return CHNS_OK;
}

}  // extern "C"
