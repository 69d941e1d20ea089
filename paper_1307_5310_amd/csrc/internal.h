// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/stdg.h"

namespace stdg {

constexpr int kMaxA = 9;   // p <= 8
constexpr int kMaxQ = 6;

// Thread-local error reporting.
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define STDG_HIP(call)                                         \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return ::stdg::hip_fail(e_, #call);  \
  } while (0)

// Element flags.
enum : int32_t {
  kAffine = 1,        // parallelepiped: constant metric
  kDiagMass = 2,      // metric diagonal (axis-aligned box)
  kPermuted = 4,      // some neighbour meets this element in another orientation
  kBoundaryBase = 8,  // bit 3 + f: face f is a PEC boundary face
  kHanging = 512,     // a face of this element is a 2:1 hanging face (ElemInfo.pad indexes HangRec)
  kHangFaceBase = 1024,  // bit 10 + f: face f is a 2:1 hanging face (either side)
  kLocalTime = 1 << 16,  // this element or a face neighbour has several temporal sub-intervals:
                         // its row runs in the local-time kernel (ElemInfo.pad indexes LTRec)
};

// Local time steps (Section 2.2): the slab interval of an element bisected
// into n = ElemInfo.nsub equal sub-intervals (a power of two, 1..kMaxSub).
// Its trial block holds 1 + n q levels (continuous piecewise P_q in time):
// level 0 the value at the slab start, level 1 the value at the slab end,
// then per sub-interval j the q levels 2 + j q .. 1 + (j + 1) q: its l_2..l_q
// and, for j < n - 1, the value at its right end (also l_0 of sub-interval
// j + 1).  Its n q test levels are L_i on sub-interval j at j q + i.
constexpr int kMaxSub = 8;
constexpr int kMaxLocalLevels = 24;  // n q <= 24 test levels
constexpr int kMaxDissLocalA7 = 5;  // D_h with local time steps and q >= 5: p + 1 <= 5
__host__ __device__ inline int local_trial_level(int q, int n, int j, int m) {
  if (m == 0) return j == 0 ? 0 : 1 + j * q;
  if (m == 1) return j == n - 1 ? 1 : 1 + (j + 1) * q;
  return 2 + j * q + m - 2;
}
// Row of an element with kLocalTime: offsets into the table bank of its own
// time tables (D[I][M] = int L_I d_s phi_M, N[I][M] = int L_I phi_M over the
// unit slab coordinate s; n q rows, 1 + n q columns) and, per face, of the
// neighbour coupling C[I][M'] = int (pi L_I) phi'_M' (pi the projection onto
// the common temporal test space of S_h, Section 4.1; 1 + n' q' columns);
// -1 on boundary faces.
struct LTRec {
  int32_t elem;
  int32_t d_off, n_off;
  int32_t c_off[6];
  int32_t s_off[6];  // D_h: own trial against the projected test function (interior faces; -1 else)
};
// Time tables of local time steps into `bank` (tables.cpp); returns the offset.
int local_time_tables(int q, int n, std::vector<double>* bank, int32_t* d_off, int32_t* n_off);
int local_coupling_table(int q, int n, int qk, int nk, std::vector<double>* bank);
int local_projected_table(int q, int n, int r, int npj, std::vector<double>* bank);

// 2:1 hanging faces (Section 5.2 sums the flux terms of a face over the
// neighbours that share parts of it): a coarse face covered by the faces of
// four smaller elements.  Per face of an element with kHanging:
//   kind 0: conforming or boundary (ElemInfo.nb / orient apply);
//   kind 1: coarse side, nb[j] covers the quarter (hu, hv) = (j & 1, j >> 1)
//           of this face, [hu/2, (hu+1)/2] x [hv/2, (hv+1)/2] in (u, v);
//   kind 2: fine side, nb[0] is the coarse element.
// code[j]: bits 0-2 the neighbour's local face; bit 3 swap (our u runs along
// the neighbour's v'); bit 4 (5): the neighbour coordinate matched with our
// u (v) runs from 1 to 0; fine side only: bit 6 (7) the half of the coarse
// face's coordinate matched with our u (v) that this face covers.
// (u, v) are the two tangential reference axes of a face in increasing order.
struct HangFace {
  int32_t kind;
  int32_t nb[4];
  uint8_t code[4];
};
struct HangRec {
  HangFace f[6];
  int32_t elem;  // the element this record belongs to
};
// 1D half-interval restriction integrals S[h][k][m] = int_0^1 L_k(x) L_m((x + h) / 2) dx
void fill_half_tables_f64(double* S);  // 2 * kMaxA * kMaxA entries

// Orientation of interior face f as seen from its element (byte orient[f]):
//   bits 0-2  the neighbour's local face f' (axis f' / 2, side f' % 2)
//   bit 3     swap: our face coordinate u runs along the neighbour's v', v along u'
//   bit 4     the neighbour coordinate matched with our u runs from 1 to 0
//   bit 5     the same for our v
// (u, v) are the two tangential reference axes of a face in increasing order.
// Canonical orientation is f' = f ^ 1 with bits 3-5 clear.
enum : uint8_t { kOrientSwap = 8, kOrientFlipU = 16, kOrientFlipV = 32 };

// Per-element record read by the kernels (64 bytes).
struct ElemInfo {
  int32_t a, q, flags, pad;
  int64_t trial_off, unk_off;
  int32_t nb[6];
  uint8_t orient[6];
  uint8_t nsub;  // temporal sub-intervals (1 = one temporal element per slab)
  uint8_t pad2;
};
static_assert(sizeof(ElemInfo) == 64, "ElemInfo layout");

// Per-element metric coefficients, FP64: symmetric 3x3 as xx, yy, zz, xy, xz, yz.
//   m[0..5]  = eps |J| DF^{-1} DF^{-T}      (mass of E, constant part)
//   m[6..11] = mu  |J| DF^{-1} DF^{-T}
//   m[12..17], m[18..23] = inverses of the two (preconditioner)
// For trilinear elements these are taken at the element centre (used by the
// preconditioner only); the mass itself is integrated from the vertices.
struct ElemMetric {
  double m[24];
  double eps, mu;  // material coefficients
};

// 1D tables passed by value to kernels (kernel-argument segment).
template <typename T>
struct Tables {
  T N[kMaxQ][kMaxQ + 1];   // N[i][m] = int_0^1 L_i l_m
  T Dh[kMaxA][kMaxA];      // Dh[n][j] = int_0^1 L_n L_j'
  T tr0[kMaxA], tr1[kMaxA];// L_j(0), L_j(1)
};

void fill_tables_f64(Tables<double>* t);
void fill_tables_f32(Tables<float>* t);

// Mass quadrature of trilinear elements: Gauss-Legendre with n = a + 1 points
// per direction on [0, 1]; B[g * a + j] = sqrt(w_g) L_j(x_g), x[g] = x_g.
template <typename T>
struct QTables {
  T B[(kMaxA + 1) * kMaxA];
  T x[kMaxA + 1];
};
void fill_qtables_f64(int a, QTables<double>* t);
void fill_qtables_f32(int a, QTables<float>* t);

// Face rule of D_h on trilinear elements: the n-point Gauss rule on [0, 1]
// (n = max(a, a') + 2 points for a face between degrees a and a') and the
// orthonormal Legendre values at its points, L[k * kMaxA + j] = L_j(x_k).
constexpr int kMaxFaceQ = kMaxA + 2;
template <typename T>
struct FaceRule {
  T x[kMaxFaceQ], w[kMaxFaceQ];
  T L[kMaxFaceQ * kMaxA];
};
void fill_face_rule_f64(int n, FaceRule<double>* r);
void fill_face_rule_f32(int n, FaceRule<float>* r);

// n-point Gauss-Legendre rule on [0, 1] (n <= 16), Newton iteration on P_n.
void gauss_rule01(int n, double* x, double* w);

// Largest q of the trilinear level-split launch variant (one workgroup per
// element and test level).
constexpr int kMaxLevelSplitQ = 4;

// Kernel work group of elements with the same (a, q, affine).
struct Group {
  int a, q, affine;
  int variant = 0;  // launch variant of the group's kernels (0..2, residual_kernel.h element_body)
  int64_t count;
  int32_t* d_list;           // element ids, locality order (device)
  std::vector<int32_t> ids;  // the same on the host
};

struct Ctx {
  int device;
  size_t budget;
  size_t used;
  // Optional device chunk that every allocation of this context is carved
  // from (a serving request's reservation): bump allocation, 256-byte
  // aligned; frees inside the chunk are no-ops, the owner returns it whole.
  char* chunk = nullptr;
  size_t chunk_size = 0, chunk_off = 0;
};

class SlabSolver;

struct Mesh {
  Ctx* ctx = nullptr;
  int64_t ne, nv;
  int64_t n_int_faces, n_bnd_faces;
  std::vector<int32_t> p, q;
  std::vector<int64_t> trial_off, unk_off, state_off;
  std::vector<ElemInfo> info;
  std::vector<ElemMetric> metric;
  std::vector<double> verts;   // [ne][8][3] element vertex coordinates
  std::vector<Group> groups;
  int n_affine, n_nonaffine, n_diag;
  int work_order = 0;  // work-list order of the groups: 0 Morton, T >= 2 columns of T x T
  // bumped by every change that captured launches would not see: D_h switched
  // on or off (its device coefficients are freed or allocated), the work lists
  // rewritten, the preconditioner scratch reallocated.  A slab solver drops
  // its captured graphs when the epoch differs from the one they were captured at.
  uint64_t epoch = 0;
  // materials and metric bounds for the iteration-error bound: min eps, min mu,
  // and max over elements of n / lambda_min(|J| DF^{-1} DF^{-T}) (centre metric; n sub-intervals)
  double eps_min = 0.0, mu_min = 0.0, inv_gmin = 0.0;
  int p_max, q_max;
  // device copies
  ElemInfo* d_info = nullptr;
  ElemMetric* d_metric = nullptr;
  double* d_verts = nullptr;
  size_t device_bytes = 0;
  int64_t* d_state_off = nullptr;
  // mass rules of trilinear elements, indexed by a (QTables<double>, QTables<float>)
  void* d_qt64 = nullptr;
  void* d_qt32 = nullptr;
  // face rules of D_h on trilinear elements, indexed by n (FaceRule<double>, FaceRule<float>)
  void* d_fr64 = nullptr;
  void* d_fr32 = nullptr;
  // 2:1 hanging faces: records of the elements with kHanging (ElemInfo.pad
  // indexes them) and the half-interval restriction tables (FP64, FP32)
  std::vector<HangRec> hang;
  int64_t n_hanging_faces = 0;  // coarse faces with four fine neighbours
  HangRec* d_hang = nullptr;
  void* d_hs64 = nullptr;
  void* d_hs32 = nullptr;
  // local time steps: sub-intervals per element, the rows of the local-time
  // kernel (elements with kLocalTime, left out of the kernel groups) and the
  // time-table bank (FP64, FP32)
  std::vector<int32_t> nsub;
  std::vector<LTRec> lt;
  std::vector<int32_t> lt_work;  // workgroups of the local-time kernel: record * kMaxSub + sub-interval,
                                 // grouped by a: lt_work[lt_a_off[a] .. lt_a_off[a + 1]) have p + 1 = a
  std::vector<int64_t> lt_a_off;
  std::vector<int32_t> lt_a_qmax;  // the largest q among the rows with p + 1 = a
  std::vector<double> lt_bank;
  LTRec* d_lt = nullptr;
  int32_t* d_lt_work = nullptr;
  void* d_ltb64 = nullptr;
  void* d_ltb32 = nullptr;
  // side streams for applies over several kernel groups (created on first use):
  // the groups run concurrently, forked from and joined back into the caller's stream
  static constexpr int kAux = 4;
  hipStream_t aux[kAux] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kAux] = {};
  // scratch for preconditioned applies on non-diagonal meshes (lazily sized)
  void* d_scratch = nullptr;
  size_t scratch_bytes = 0;
  // dissipative stabilisation D_h (c = 0: off): per element kDissWords doubles,
  //   [g]      alpha_E of face g        [6 + g]  alpha_H of face g (0 on PEC faces)
  //   [12 + 3 alpha + (0, 1, 2)] = K_aa, K_bb, K_ab of the faces normal to alpha,
  // K = |t_a x t_b| g^{-1} the face metric of the tangent vectors t_a, t_b along
  // the axes (alpha + 1) % 3, (alpha + 2) % 3 (constant on affine elements;
  // unused on trilinear ones, whose kernel evaluates it at the face points)
  // the slab solver of stdg_slab_solve, kept between calls (its Krylov basis
  // and work vectors stay allocated: a march of slabs allocates once); a call
  // that finds it busy (another thread) uses a solver of its own
  SlabSolver* solver = nullptr;
  std::atomic<bool> solver_busy{false};
  static constexpr int kDissWords = 24;
  double c_diss = 0.0;
  double* d_diss = nullptr;   // FP64 copy (FP64 kernels)
  float* d_diss32 = nullptr;  // FP32 copy (FP32 kernels)
};

// Kernel launchers (residual.hip).
struct ApplyArgs {
  const Mesh* mesh;
  double dt;
  int prec;
  int mode;
  const void* x;
  const void* load;
  void* y;
  hipStream_t stream;
  // the allocation-free variant: the preconditioner pre-pass uses the static
  // device scratch, and several kernel groups run one after another on
  // `stream` (no side streams or events are created)
  bool no_alloc = false;
  // device flag read by the kernels at entry: 0 = return at once (kernels of
  // Arnoldi iterations past the end of a restart cycle); NULL = always run
  const int* skip = nullptr;
};
int launch_residual(const ApplyArgs& a);
// per-element W_h' dual norms (both fields) of a residual-layout FP64 vector on
// the trilinear elements, into partial[2 e], partial[2 e + 1] (dualnorm.hip)
int launch_dual_norm_trilinear(const Mesh* m, const double* R, double* partial, hipStream_t s);
// Static device scratch of the allocation-free apply: look up this device's
// address of the array (once per device; the device must be current).
int noalloc_scratch_init(int device);
size_t noalloc_scratch_capacity();
int launch_precond_scale(const Mesh* m, int prec, const void* x, void* z, hipStream_t s, const int* skip = nullptr);
// the same on meshes with local time steps (also the sub-interval time factor; local_time.hip)
int launch_precond_scale_local(const Mesh* m, int prec, const void* x, void* z, hipStream_t s, const int* skip);
// One request's operands of a batched preconditioned operator apply (the
// serving loop's lockstep restart cycles; residual.hip).
struct BatchApplyArgs {
  const Mesh* mesh;
  double dt;
  const void* x;
  void* y;
  const int* skip;
};
// a mesh that can join batched applies: one affine kernel group, a diagonal
// metric (P^{-1} fused into the kernel), no D_h
bool batchable_mesh(const Mesh* m);
// up to 16 requests whose meshes are batchable with the same (a, q)
int launch_residual_batch(const BatchApplyArgs* a, int count, int prec, hipStream_t s);
// bytes (a multiple of 16) from src to dst, both 16-byte aligned, no overlap (blas.hip)
int stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
// the neighbours' half of the centred flux on 2:1 hanging faces, added to y
// after the residual kernels (hanging.hip); any mode (P^{-1} fused on
// diagonal meshes, else x already scaled and mode 0)
template <typename T>
int launch_hanging(const Mesh* m, double dt, int mode, const T* x, T* y, hipStream_t s, const int* skip);
// the rows of the elements with kLocalTime, written to y (local_time.hip);
// mode 0 or STDG_RESIDUAL (preconditioned applies take the P^{-1} pre-pass)
template <typename T>
int launch_local_time(const Mesh* m, double dt, int mode, const T* x, const T* load, T* y, hipStream_t s,
                      const int* skip);
// D_h on the trilinear group g, added to y (dissipation.hip); mode 0 or STDG_RESIDUAL
template <typename T>
int launch_diss_trilinear(const Mesh* m, const Group& g, double dt, int mode, const T* x, T* y, hipStream_t s,
                          const int* skip);

// Mesh construction (mesh.cpp): host analysis (validation, faces, metric,
// groups) and the device copies, separable so that a server can analyse a
// request's mesh on the submitting thread.
int build_mesh_host(const stdg_mesh_desc* d, Mesh* m);
int upload_mesh(Ctx* ctx, Mesh* m);
int build_mesh(Ctx* ctx, const stdg_mesh_desc* d, Mesh* m);
void release_mesh(Mesh* m);
size_t mesh_device_bytes(const Mesh& m);
int set_dissipation(Mesh* m, double c);
int default_work_order(const Mesh& m);
int set_work_order(Mesh* m, int order);  // host lists, and the device lists once uploaded
void release_cached_solver(Mesh* m);  // solver.cpp

// Allocation against the context budget.
int dev_alloc(Ctx* ctx, void** p, size_t bytes);
void dev_free(Ctx* ctx, void* p, size_t bytes);

}  // namespace stdg

struct stdg_ctx { stdg::Ctx c; };
struct stdg_mesh { stdg::Mesh m; };
