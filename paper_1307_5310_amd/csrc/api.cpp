// C-ABI entry points: contexts, errors, meshes, and the residual apply.
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

namespace stdg {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const std::string& msg) {
  set_error(msg);
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " + what);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return STDG_E_NOMEM;
  return STDG_E_DEVICE;
}

int dev_alloc(Ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (ctx->chunk) {
    const size_t off = (ctx->chunk_off + 255) & ~(size_t)255;
    if (off + bytes > ctx->chunk_size)
      return fail(STDG_E_CAPACITY, "allocation of " + std::to_string(bytes) + " bytes exceeds the reservation (" +
                                       std::to_string(off) + " of " + std::to_string(ctx->chunk_size) + " used)");
    *p = ctx->chunk + off;
    ctx->chunk_off = off + bytes;
    ctx->used += bytes;
    return STDG_OK;
  }
  if (ctx->used + bytes > ctx->budget)
    return fail(STDG_E_CAPACITY, "allocation of " + std::to_string(bytes) + " bytes exceeds the HBM budget (" +
                                     std::to_string(ctx->used) + " of " + std::to_string(ctx->budget) + " used)");
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(e, "hipMalloc");
  }
  ctx->used += bytes;
  return STDG_OK;
}

void dev_free(Ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  if (bytes == 0) bytes = 256;
  const bool in_chunk = ctx->chunk && (char*)p >= ctx->chunk && (char*)p < ctx->chunk + ctx->chunk_size;
  if (!in_chunk) (void)hipFree(p);
  ctx->used = ctx->used >= bytes ? ctx->used - bytes : 0;
}

int build_mesh(Ctx* ctx, const stdg_mesh_desc* d, Mesh* m);
void release_mesh(Mesh* m);

}  // namespace stdg

using namespace stdg;

extern "C" {

int stdg_version(void) { return (1 << 16) | 1; }

size_t stdg_struct_size(int32_t which) {
  switch (which) {
    case STDG_STRUCT_MESH_DESC: return sizeof(stdg_mesh_desc);
    case STDG_STRUCT_MESH_INFO: return sizeof(stdg_mesh_info_t);
    case STDG_STRUCT_SOURCE: return sizeof(stdg_source);
    case STDG_STRUCT_SOLVE_OPTS: return sizeof(stdg_solve_opts);
    case STDG_STRUCT_SOLVE_INFO: return sizeof(stdg_solve_info);
    case STDG_STRUCT_SERVE_OPTS: return sizeof(stdg_serve_opts);
    case STDG_STRUCT_REQUEST: return sizeof(stdg_request);
    case STDG_STRUCT_RESULT: return sizeof(stdg_result);
    case STDG_STRUCT_GROUP_INFO: return sizeof(stdg_group_info_t);
    default: return 0;
  }
}

const char* stdg_last_error(void) { return g_last_error.c_str(); }

int stdg_init(int hip_device, size_t hbm_budget_bytes, stdg_ctx** out) {
  if (!out) return fail(STDG_E_ARG, "stdg_init: out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) return fail(STDG_E_DEVICE, "stdg_init: no HIP device available");
  if (hip_device < 0 || hip_device >= n) return fail(STDG_E_ARG, "stdg_init: device index out of range");
  STDG_HIP(hipSetDevice(hip_device));
  hipDeviceProp_t prop;
  STDG_HIP(hipGetDeviceProperties(&prop, hip_device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(STDG_E_DEVICE, std::string("stdg_init: built for gfx950, device is ") + prop.gcnArchName);
  size_t free_b = 0, total_b = 0;
  STDG_HIP(hipMemGetInfo(&free_b, &total_b));
  stdg_ctx* c = new (std::nothrow) stdg_ctx;
  if (!c) return fail(STDG_E_NOMEM, "stdg_init: host allocation failed");
  // this device's address of the static scratch of stdg_residual_apply_noalloc
  int rc = noalloc_scratch_init(hip_device);
  if (rc != STDG_OK) {
    delete c;
    return rc;
  }
  c->c.device = hip_device;
  c->c.budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
  c->c.used = 0;
  *out = c;
  return STDG_OK;
}

int stdg_finalize(stdg_ctx* ctx) {
  if (!ctx) return fail(STDG_E_ARG, "stdg_finalize: ctx is NULL");
  delete ctx;
  return STDG_OK;
}

int stdg_mesh_upload(stdg_ctx* ctx, const stdg_mesh_desc* desc, stdg_mesh** out) {
  if (!ctx || !desc || !out) return fail(STDG_E_ARG, "stdg_mesh_upload: NULL argument");
  *out = nullptr;
  if (desc->n_elements <= 0 || desc->n_vertices <= 0 || !desc->vertices || !desc->hexes || !desc->p ||
      !desc->q || !desc->eps || !desc->mu)
    return fail(STDG_E_ARG, "stdg_mesh_upload: empty mesh or NULL array");
  if (desc->n_elements > (int64_t)INT32_MAX) return fail(STDG_E_ARG, "stdg_mesh_upload: too many elements");
  STDG_HIP(hipSetDevice(ctx->c.device));
  stdg_mesh* m = new (std::nothrow) stdg_mesh;
  if (!m) return fail(STDG_E_NOMEM, "stdg_mesh_upload: host allocation failed");
  int rc;
  try {
    rc = build_mesh(&ctx->c, desc, &m->m);
  } catch (const std::bad_alloc&) {
    rc = fail(STDG_E_NOMEM, "stdg_mesh_upload: host allocation failed");
  }
  if (rc != STDG_OK) {
    release_mesh(&m->m);
    delete m;
    return rc;
  }
  *out = m;
  return STDG_OK;
}

int stdg_mesh_info(const stdg_mesh* mesh, stdg_mesh_info_t* out) {
  if (!mesh || !out) return fail(STDG_E_ARG, "stdg_mesh_info: NULL argument");
  const Mesh& m = mesh->m;
  std::memset(out, 0, sizeof(*out));
  out->n_elements = m.ne;
  out->n_vertices = m.nv;
  out->n_interior_faces = m.n_int_faces;
  out->n_boundary_faces = m.n_bnd_faces;
  out->trial_size = m.trial_off.back();
  out->unknown_size = m.unk_off.back();
  out->state_size = m.state_off.back();
  out->n_groups = (int32_t)m.groups.size();
  out->n_affine = m.n_affine;
  out->n_nonaffine = m.n_nonaffine;
  out->n_diagonal_mass = m.n_diag;
  out->p_max = m.p_max;
  out->q_max = m.q_max;
  out->device_bytes = (int64_t)m.device_bytes;
  out->work_order = m.work_order;
  return STDG_OK;
}

int stdg_mesh_offsets(const stdg_mesh* mesh, int64_t* trial_off, int64_t* unknown_off, int64_t* state_off) {
  if (!mesh) return fail(STDG_E_ARG, "stdg_mesh_offsets: mesh is NULL");
  const Mesh& m = mesh->m;
  size_t n = sizeof(int64_t) * (m.ne + 1);
  if (trial_off) std::memcpy(trial_off, m.trial_off.data(), n);
  if (unknown_off) std::memcpy(unknown_off, m.unk_off.data(), n);
  if (state_off) std::memcpy(state_off, m.state_off.data(), n);
  return STDG_OK;
}

int stdg_mesh_set_order(stdg_mesh* mesh, int32_t order) {
  if (!mesh) return fail(STDG_E_ARG, "stdg_mesh_set_order: mesh is NULL");
  return stdg::set_work_order(&mesh->m, order);
}

int stdg_mesh_set_launch(stdg_mesh* mesh, int32_t group, int32_t variant) {
  if (!mesh) return fail(STDG_E_ARG, "stdg_mesh_set_launch: mesh is NULL");
  Mesh* m = &mesh->m;
  if (variant < 0 || variant > 2) return fail(STDG_E_ARG, "stdg_mesh_set_launch: variant must be 0, 1 or 2");
  if (group < -1 || group >= (int32_t)m->groups.size()) return fail(STDG_E_ARG, "stdg_mesh_set_launch: no such group");
  for (int32_t k = 0; k < (int32_t)m->groups.size(); ++k) {
    if (group >= 0 && k != group) continue;
    Group& g = m->groups[k];
    // affine groups: variants 0..2; trilinear groups: 0, or 1 when 1 < q <= 4
    // (any other request is taken as 0)
    g.variant = g.affine ? variant : (variant == 1 && g.q > 1 && g.q <= kMaxLevelSplitQ ? 1 : 0);
  }
  ++m->epoch;  // captured launches carry the old variant
  return STDG_OK;
}

int stdg_mesh_group(const stdg_mesh* mesh, int32_t group, stdg_group_info_t* out) {
  if (!mesh || !out) return fail(STDG_E_ARG, "stdg_mesh_group: NULL argument");
  const Mesh& m = mesh->m;
  if (group < 0 || group >= (int32_t)m.groups.size()) return fail(STDG_E_ARG, "stdg_mesh_group: no such group");
  const Group& g = m.groups[group];
  out->p = g.a - 1;
  out->q = g.q;
  out->affine = g.affine;
  out->variant = g.variant;
  out->n_elements = g.count;
  return STDG_OK;
}

int stdg_mesh_autotune(stdg_mesh* mesh, int prec, double dt, int32_t reps, int32_t* order_out, void* stream) {
  if (!mesh || !order_out) return fail(STDG_E_ARG, "stdg_mesh_autotune: NULL argument");
  if (prec != STDG_FP64 && prec != STDG_FP32) return fail(STDG_E_ARG, "stdg_mesh_autotune: unknown precision");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(STDG_E_ARG, "stdg_mesh_autotune: dt must be finite and > 0");
  if (reps < 1) reps = 10;
  Mesh* m = &mesh->m;
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)m->unk_off.back() * (prec == STDG_FP64 ? 8 : 4);
  void *x = nullptr, *y = nullptr;
  int rc = dev_alloc(m->ctx, &x, bytes);
  if (rc == STDG_OK) rc = dev_alloc(m->ctx, &y, bytes);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (rc == STDG_OK && hipEventCreate(&e0) != hipSuccess) rc = fail(STDG_E_DEVICE, "stdg_mesh_autotune: event");
  if (rc == STDG_OK && hipEventCreate(&e1) != hipSuccess) rc = fail(STDG_E_DEVICE, "stdg_mesh_autotune: event");
  if (rc == STDG_OK && hipMemsetAsync(x, 0, bytes, s) != hipSuccess) rc = fail(STDG_E_DEVICE, "stdg_mesh_autotune: memset");
  ApplyArgs a{m, dt, prec, STDG_OPERATOR_PRECOND, x, nullptr, y, s};
  // milliseconds for `reps` preconditioned applies after two untimed ones
  auto time_applies = [&](float* ms) -> int {
    int r = STDG_OK;
    for (int w = 0; w < 2 && r == STDG_OK; ++w) r = launch_residual(a);
    if (r != STDG_OK) return r;
    if (hipEventRecord(e0, s) != hipSuccess) return fail(STDG_E_DEVICE, "stdg_mesh_autotune: event");
    for (int k = 0; k < reps && r == STDG_OK; ++k) r = launch_residual(a);
    if (r != STDG_OK) return r;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return fail(STDG_E_DEVICE, "stdg_mesh_autotune: timing");
    return STDG_OK;
  };
  // untimed applies first, so that the GPU's clocks have risen before the
  // first candidate is timed
  for (int w = 0; w < 10 * reps && rc == STDG_OK; ++w) rc = launch_residual(a);
  // (1) the work-list order, every group in its current variant
  const int candidates[4] = {0, 4, 8, 16};
  int best = m->work_order;
  float best_ms = 0.0f;
  for (int k = 0; k < 4 && rc == STDG_OK; ++k) {
    if ((rc = set_work_order(m, candidates[k])) != STDG_OK) break;
    float ms = 0.0f;
    if ((rc = time_applies(&ms)) != STDG_OK) break;
    if (k == 0 || ms < best_ms) {
      best_ms = ms;
      best = candidates[k];
    }
  }
  if (rc == STDG_OK) rc = set_work_order(m, best);
  // (2) each affine group's launch variant, with the order chosen and the
  // other groups in their current variants
  for (size_t gi = 0; gi < m->groups.size() && rc == STDG_OK; ++gi) {
    Group& g = m->groups[gi];
    if (g.count == 0) continue;
    int vbest = g.variant;
    float vms = 0.0f;
    const int nvar = g.affine ? 3 : (g.q > 1 && g.q <= kMaxLevelSplitQ ? 2 : 1);
    for (int v = 0; v < nvar && rc == STDG_OK; ++v) {
      g.variant = v;
      float ms = 0.0f;
      if ((rc = time_applies(&ms)) != STDG_OK) break;
      if (v == 0 || ms < vms) {
        vms = ms;
        vbest = v;
      }
    }
    g.variant = vbest;
  }
  if (s) (void)hipStreamSynchronize(s); else (void)hipDeviceSynchronize();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (x) dev_free(m->ctx, x, bytes);
  if (y) dev_free(m->ctx, y, bytes);
  if (rc != STDG_OK) return rc;
  ++m->epoch;  // launch variants changed under any captured launches
  *order_out = best;
  return STDG_OK;
}

int stdg_mesh_set_dissipation(stdg_mesh* mesh, double c) {
  if (!mesh) return fail(STDG_E_ARG, "stdg_mesh_set_dissipation: mesh is NULL");
  STDG_HIP(hipSetDevice(mesh->m.ctx->device));
  return stdg::set_dissipation(&mesh->m, c);
}

int stdg_mesh_free(stdg_mesh* mesh) {
  if (!mesh) return fail(STDG_E_ARG, "stdg_mesh_free: mesh is NULL");
  release_mesh(&mesh->m);
  delete mesh;
  return STDG_OK;
}

int stdg_residual_apply(const stdg_mesh* mesh, double dt, int prec, int mode, const void* x_dev,
                        const void* load_dev, void* y_dev, void* stream) {
  if (!mesh) return fail(STDG_E_ARG, "stdg_residual_apply: mesh is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(STDG_E_ARG, "stdg_residual_apply: dt must be finite and > 0");
  if (prec != STDG_FP64 && prec != STDG_FP32) return fail(STDG_E_ARG, "stdg_residual_apply: unknown precision");
  if (mode != STDG_OPERATOR && mode != STDG_RESIDUAL && mode != STDG_OPERATOR_PRECOND)
    return fail(STDG_E_ARG, "stdg_residual_apply: unknown mode");
  if (!x_dev || !y_dev) return fail(STDG_E_ARG, "stdg_residual_apply: x or y is NULL");
  if (load_dev && mode != STDG_RESIDUAL) return fail(STDG_E_ARG, "stdg_residual_apply: load only in RESIDUAL mode");
  if (x_dev == y_dev) return fail(STDG_E_ARG, "stdg_residual_apply: x and y must not alias");
  ApplyArgs a{&mesh->m, dt, prec, mode, x_dev, load_dev, y_dev, (hipStream_t)stream};
  return launch_residual(a);
}

int stdg_residual_apply_noalloc(const stdg_mesh* mesh, double dt, int prec, int mode, const void* x_dev,
                                const void* load_dev, void* y_dev, void* stream) {
  if (!mesh) return fail(STDG_E_ARG, "stdg_residual_apply_noalloc: mesh is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(STDG_E_ARG, "stdg_residual_apply_noalloc: dt must be finite and > 0");
  if (prec != STDG_FP64 && prec != STDG_FP32) return fail(STDG_E_ARG, "stdg_residual_apply_noalloc: unknown precision");
  if (mode != STDG_OPERATOR && mode != STDG_RESIDUAL && mode != STDG_OPERATOR_PRECOND)
    return fail(STDG_E_ARG, "stdg_residual_apply_noalloc: unknown mode");
  if (!x_dev || !y_dev) return fail(STDG_E_ARG, "stdg_residual_apply_noalloc: x or y is NULL");
  if (load_dev && mode != STDG_RESIDUAL)
    return fail(STDG_E_ARG, "stdg_residual_apply_noalloc: load only in RESIDUAL mode");
  if (x_dev == y_dev) return fail(STDG_E_ARG, "stdg_residual_apply_noalloc: x and y must not alias");
  ApplyArgs a{&mesh->m, dt, prec, mode, x_dev, load_dev, y_dev, (hipStream_t)stream};
  a.no_alloc = true;
  return launch_residual(a);
}

size_t stdg_noalloc_scratch_bytes(void) { return noalloc_scratch_capacity(); }

int stdg_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (bytes == 0) return STDG_OK;
  if (!src || !dst) return fail(STDG_E_ARG, "stdg_stream_copy: NULL buffer");
  if (bytes % 16 != 0 || (uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0)
    return fail(STDG_E_ARG, "stdg_stream_copy: buffers and size must be multiples of 16 bytes");
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
  if (a < b + bytes && b < a + bytes) return fail(STDG_E_ARG, "stdg_stream_copy: buffers overlap");
  return stream_copy(src, dst, bytes, (hipStream_t)stream);
}

}  // extern "C"
