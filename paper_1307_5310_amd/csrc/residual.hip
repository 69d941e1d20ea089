// Dispatch of the residual kernels over the (a, q, affine) groups of a mesh.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "residual_kernel.h"

namespace stdg {

// Device scratch of stdg_residual_apply_noalloc, for callers that cannot
// allocate: the P^{-1} pre-pass of preconditioned applies on meshes with a
// non-diagonal metric writes the scaled input here instead of into the
// mesh's lazily allocated scratch.  Each device holds its own copy until the
// process ends.  In host code the array's name is not a device address: host
// code uses only the address hipGetSymbolAddress returned for the current
// device (kept per device below).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t noalloc_scratch_capacity() { return kNoAllocScratchBytes; }

int noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(STDG_E_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return STDG_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
  g_scratch_ptr[device] = ptr;
  return STDG_OK;
}

static void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

#define STDG_DECL(K, R, AA) int launch_##K##R##AA(int q, const KParams<R>& P, int64_t n, hipStream_t s);
#define STDG_DECL_ALL(K, R) STDG_DECL(K, R, 2) STDG_DECL(K, R, 3) STDG_DECL(K, R, 4) STDG_DECL(K, R, 5) \
  STDG_DECL(K, R, 6) STDG_DECL(K, R, 7) STDG_DECL(K, R, 8) STDG_DECL(K, R, 9)
STDG_DECL_ALL(affine_, float)
STDG_DECL_ALL(affine_, double)
STDG_DECL_ALL(trilinear_, float)
STDG_DECL_ALL(trilinear_, double)
STDG_DECL_ALL(affine_diss_, float)
STDG_DECL_ALL(affine_diss_, double)
#undef STDG_DECL_ALL
#undef STDG_DECL

#define STDG_BDECL(R, AA) int launch_batch_##R##AA(int q, const BatchKParams<R>& B, uint32_t total, hipStream_t s);
#define STDG_BDECL_ALL(R) STDG_BDECL(R, 2) STDG_BDECL(R, 3) STDG_BDECL(R, 4) STDG_BDECL(R, 5) STDG_BDECL(R, 6) \
  STDG_BDECL(R, 7) STDG_BDECL(R, 8) STDG_BDECL(R, 9)
STDG_BDECL_ALL(float)
STDG_BDECL_ALL(double)
#undef STDG_BDECL_ALL
#undef STDG_BDECL

template <typename T>
using Launcher = int (*)(int, const KParams<T>&, int64_t, hipStream_t);
template <typename T>
using BatchLauncher = int (*)(int, const BatchKParams<T>&, uint32_t, hipStream_t);
static BatchLauncher<float> batch_f32[kMaxA + 1] = {nullptr, nullptr, launch_batch_float2, launch_batch_float3,
                                                    launch_batch_float4, launch_batch_float5, launch_batch_float6,
                                                    launch_batch_float7, launch_batch_float8, launch_batch_float9};
static BatchLauncher<double> batch_f64[kMaxA + 1] = {nullptr, nullptr, launch_batch_double2, launch_batch_double3,
                                                     launch_batch_double4, launch_batch_double5, launch_batch_double6,
                                                     launch_batch_double7, launch_batch_double8, launch_batch_double9};
static_assert(kMaxApplyBatch >= 16, "batched applies hold the serving loop's batches");

#define STDG_TABLE(K, R) \
  { nullptr, nullptr, launch_##K##R##2, launch_##K##R##3, launch_##K##R##4, launch_##K##R##5, \
    launch_##K##R##6, launch_##K##R##7, launch_##K##R##8, launch_##K##R##9 }
static Launcher<float> affine_f32[kMaxA + 1] = STDG_TABLE(affine_, float);
static Launcher<double> affine_f64[kMaxA + 1] = STDG_TABLE(affine_, double);
static Launcher<float> trilinear_f32[kMaxA + 1] = STDG_TABLE(trilinear_, float);
static Launcher<double> trilinear_f64[kMaxA + 1] = STDG_TABLE(trilinear_, double);
static Launcher<float> affine_diss_f32[kMaxA + 1] = STDG_TABLE(affine_diss_, float);
static Launcher<double> affine_diss_f64[kMaxA + 1] = STDG_TABLE(affine_diss_, double);
#undef STDG_TABLE

static int ensure_aux(Mesh* m) {
  if (m->fork_ev) return STDG_OK;
  for (int k = 0; k < Mesh::kAux; ++k) {
    STDG_HIP(hipStreamCreateWithFlags(&m->aux[k], hipStreamNonBlocking));
    STDG_HIP(hipEventCreateWithFlags(&m->join_ev[k], hipEventDisableTiming));
  }
  STDG_HIP(hipEventCreateWithFlags(&m->fork_ev, hipEventDisableTiming));
  return STDG_OK;
}

// Launch every (a, q, affine) group; with several groups they run on side
// streams, largest first, forked from and joined back into s (the groups
// write disjoint outputs, so the result does not depend on their order).
template <typename T>
static int run_groups(const Mesh* m, double dt, int mode, const T* x, const T* load, T* y, hipStream_t s,
                      Launcher<T>* affine, Launcher<T>* trilinear, const QTables<T>* d_qt, bool allow_fork,
                      const int* skip) {
  KParams<T> P;
  P.skip = skip;
  P.info = m->d_info;
  P.metric = m->d_metric;
  P.x = x;
  P.load = load;
  P.y = y;
  P.verts = m->d_verts;
  if constexpr (sizeof(T) == 8) P.diss = m->d_diss; else P.diss = m->d_diss32;
  P.dt = (T)dt;
  P.mode = mode;
  if constexpr (sizeof(T) == 8) fill_tables_f64(&P.tab); else fill_tables_f32(&P.tab);
  std::vector<const Group*> order;
  for (const Group& g : m->groups) {
    if (g.count == 0) continue;
    if (!g.affine && mode == STDG_OPERATOR_PRECOND)
      return fail(STDG_E_UNSUPPORTED, "trilinear elements take P^{-1} in a separate pass");
    order.push_back(&g);
  }
  auto work = [](const Group* g) { return g->count * (int64_t)g->q * g->a * g->a * g->a * (g->affine ? 1 : 3); };
  std::stable_sort(order.begin(), order.end(), [&](const Group* l, const Group* r) { return work(l) > work(r); });
  const bool fork = allow_fork && order.size() > 1;
  if (fork) {
    int rc = ensure_aux(const_cast<Mesh*>(m));
    if (rc != STDG_OK) return rc;
    STDG_HIP(hipEventRecord(m->fork_ev, s));
    for (int k = 0; k < Mesh::kAux && k < (int)order.size(); ++k) STDG_HIP(hipStreamWaitEvent(m->aux[k], m->fork_ev, 0));
  }
  for (size_t i = 0; i < order.size(); ++i) {
    const Group& g = *order[i];
    P.list = g.d_list;
    P.variant = g.variant;
    P.qt = d_qt + g.a;
    const hipStream_t gs = fork ? m->aux[i % Mesh::kAux] : s;
    int rc = (g.affine ? affine : trilinear)[g.a](g.q, P, g.count, gs);
    if (rc != STDG_OK) return rc;
    // D_h on trilinear elements: added by its own kernel after the group's residual
    if (!g.affine && m->d_diss) {
      rc = launch_diss_trilinear<T>(m, g, dt, mode, x, y, gs, skip);
      if (rc != STDG_OK) return rc;
    }
  }
  if (fork) {
    for (int k = 0; k < Mesh::kAux && k < (int)order.size(); ++k) {
      STDG_HIP(hipEventRecord(m->join_ev[k], m->aux[k]));
      STDG_HIP(hipStreamWaitEvent(s, m->join_ev[k], 0));
    }
  }
  // 2:1 hanging faces: the neighbours' half of their fluxes, after every group
  if (!m->hang.empty()) return launch_hanging<T>(m, dt, mode, x, y, s, skip);
  // local time steps: the rows left out of the groups
  if (!m->lt.empty()) return launch_local_time<T>(m, dt, mode, x, load, y, s, skip);
  return STDG_OK;
}

bool batchable_mesh(const Mesh* m) {
  int groups = 0;
  const Group* g0 = nullptr;
  for (const Group& g : m->groups)
    if (g.count > 0) {
      ++groups;
      g0 = &g;
    }
  return groups == 1 && g0->affine && m->n_diag == m->ne && m->d_diss == nullptr && m->hang.empty() &&
         m->lt.empty();
}

template <typename T>
static int run_batch(const BatchApplyArgs* a, int count, hipStream_t s, BatchLauncher<T>* table) {
  if (count < 1 || count > kMaxApplyBatch) return fail(STDG_E_ARG, "batched apply: 1 to 16 requests");
  BatchKParams<T> B;
  std::memset(&B, 0, sizeof(B));
  const Group* g0 = nullptr;
  uint64_t first = 0;
  for (int i = 0; i < count; ++i) {
    const Mesh* m = a[i].mesh;
    if (!batchable_mesh(m)) return fail(STDG_E_ARG, "batched apply: mesh not batchable");
    const Group* g = nullptr;
    for (const Group& gg : m->groups)
      if (gg.count > 0) g = &gg;
    if (g0 && (g->a != g0->a || g->q != g0->q)) return fail(STDG_E_ARG, "batched apply: degrees differ");
    g0 = g;
    BatchMember<T>& M = B.m[i];
    M.info = m->d_info;
    M.metric = m->d_metric;
    M.list = g->d_list;
    M.x = (const T*)a[i].x;
    M.y = (T*)a[i].y;
    M.skip = a[i].skip;
    M.dt = (T)a[i].dt;
    M.first = (uint32_t)first;
    first += (uint64_t)g->count;
  }
  if (first > 0xffffffffu) return fail(STDG_E_ARG, "batched apply: too many elements");
  B.count = count;
  if constexpr (sizeof(T) == 8) fill_tables_f64(&B.tab); else fill_tables_f32(&B.tab);
  return table[g0->a](g0->q, B, (uint32_t)first, s);
}

int launch_residual_batch(const BatchApplyArgs* a, int count, int prec, hipStream_t s) {
  return prec == STDG_FP64 ? run_batch<double>(a, count, s, batch_f64) : run_batch<float>(a, count, s, batch_f32);
}

int launch_precond_scale(const Mesh* m, int prec, const void* x, void* z, hipStream_t s, const int* skip) {
  if (!m->lt.empty()) return launch_precond_scale_local(m, prec, x, z, s, skip);
  const dim3 grid((unsigned)m->ne), block(256);
  if (prec == STDG_FP64)
    hipLaunchKernelGGL(precond_scale_kernel<double>, grid, block, 0, s, m->d_info, m->d_metric, m->ne,
                       (const double*)x, (double*)z, skip);
  else
    hipLaunchKernelGGL(precond_scale_kernel<float>, grid, block, 0, s, m->d_info, m->d_metric, m->ne,
                       (const float*)x, (float*)z, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "precond_scale launch");
  return STDG_OK;
}

int launch_residual(const ApplyArgs& a) {
  const Mesh* m = a.mesh;
  int mode = a.mode;
  const void* x = a.x;
  // P^{-1} as a pre-pass: on meshes with a non-diagonal metric somewhere, and
  // with local time steps (P^{-1} then also mixes the time levels)
  const bool prepass = m->n_diag != m->ne || !m->lt.empty();
  if (mode == STDG_OPERATOR_PRECOND && prepass && a.no_alloc) {
    // the allocation-free variant: P^{-1} x into the static scratch of this device
    const size_t need = (size_t)m->unk_off.back() * (a.prec == STDG_FP64 ? 8 : 4);
    if (need > kNoAllocScratchBytes)
      return fail(STDG_E_CAPACITY, "stdg_residual_apply_noalloc: the scaled input needs " + std::to_string(need) +
                                       " bytes of scratch, the static scratch holds " +
                                       std::to_string(kNoAllocScratchBytes));
    int dev = -1;
    STDG_HIP(hipGetDevice(&dev));
    int rc = noalloc_scratch_init(dev);
    if (rc != STDG_OK) return rc;
    void* ptr = noalloc_scratch(dev);
    rc = launch_precond_scale(m, a.prec, x, ptr, a.stream, a.skip);
    if (rc != STDG_OK) return rc;
    x = ptr;
    mode = STDG_OPERATOR;
  } else if (mode == STDG_OPERATOR_PRECOND && prepass) {
    // non-diagonal metric somewhere: scale into the mesh's scratch, then plain
    // operator.  The scratch is sized for FP64 on first use, so a later call in
    // the other precision never moves it under captured launches; the epoch is
    // bumped all the same should it ever be (re)allocated.
    Mesh* mm = const_cast<Mesh*>(m);
    const size_t need = (size_t)m->unk_off.back() * sizeof(double);
    if (mm->scratch_bytes < need) {
      if (mm->d_scratch) dev_free(mm->ctx, mm->d_scratch, mm->scratch_bytes);
      mm->d_scratch = nullptr;
      mm->scratch_bytes = 0;
      ++mm->epoch;
      int rc = dev_alloc(mm->ctx, &mm->d_scratch, need);
      if (rc != STDG_OK) return rc;
      mm->scratch_bytes = need;
    }
    int rc = launch_precond_scale(m, a.prec, x, mm->d_scratch, a.stream, a.skip);
    if (rc != STDG_OK) return rc;
    x = mm->d_scratch;
    mode = STDG_OPERATOR;
  }
  const bool diss = m->d_diss != nullptr;
  if (a.prec == STDG_FP64)
    return run_groups<double>(m, a.dt, mode, (const double*)x, (const double*)a.load, (double*)a.y, a.stream,
                              diss ? affine_diss_f64 : affine_f64, trilinear_f64, (const QTables<double>*)m->d_qt64,
                              !a.no_alloc, a.skip);
  return run_groups<float>(m, a.dt, mode, (const float*)x, (const float*)a.load, (float*)a.y, a.stream,
                           diss ? affine_diss_f32 : affine_f32, trilinear_f32, (const QTables<float>*)m->d_qt32,
                           !a.no_alloc, a.skip);
}

}  // namespace stdg
