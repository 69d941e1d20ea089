/*
 * stdg: space-time hp-DG residual of the time-dependent Maxwell equations on
 * one AMD MI355X (gfx950).  C ABI.
 *
 * Method: Lilienthal, Schnepp, Weiland, "Non-dissipative space-time
 * hp-discontinuous Galerkin method for the time-dependent Maxwell equations"
 * (arXiv 1307.5310).  The problem is eq. (maxwell) of Section 1 with PEC walls
 * (n x E = 0, g = 0); one time slab I_n = (t_{n-1}, t_n] at a time (Section 2.2)
 * with one temporal element per slab; local spaces of eq. (spaces:local):
 * trial P_q (time) x [Q_p]^3, test P_{q-1} x [Q_p]^3; covariant element maps
 * (Section 2.3); the slab form B_h = C_h + S_h of Section 2.5 / 4.1 with
 * centred fluxes; the residual R_h(V) = B_h(U_h, V) - L(V) of Section 5
 * (eq. residual); the bases of Section 5.1.
 *
 * Conventions used by every call
 * ------------------------------
 * Status: every function returns 0 (STDG_OK) or a negative stdg_status; the
 * message of the last failure on the calling thread is stdg_last_error().
 * No exception crosses this ABI.
 *
 * Element vertex order: local vertex v = b0 + 2 b1 + 4 b2 sits at reference
 * corner (b0, b1, b2) of [0,1]^3 (x-hat fastest).  Local face 2*alpha + side
 * lies on x-hat_alpha = side.
 *
 * Coefficient layouts (element-major in mesh order, FP32 or FP64):
 *   a = p + 1, s = j + a*(k + a*l) with (j, k, l) the Legendre degrees in
 *   (x-hat, y-hat, z-hat); field 0 = E, 1 = H; comp 0..2 = reference
 *   component c of the covariant pull-back E-hat = DF^T E o F.
 *   full trial U : per element [field][comp][m = 0..q][s], 6(q+1)a^3 scalars,
 *                  m the integrated-Legendre time level l_m (eq. def:ilegendre)
 *   unknowns x   : per element [field][comp][m = 1..q][s], 6 q a^3 scalars
 *   residual y   : per element [field][comp][i = 0..q-1][s], 6 q a^3 scalars,
 *                  i the orthonormal-Legendre test level L_i
 *   state        : per element [field][comp][s], 6 a^3 scalars (fields at one
 *                  time; the l_0 block of a slab is the state at its start and
 *                  the l_1 block the state at its end)
 * Element offsets are prefix sums of these sizes (stdg_mesh_offsets).
 *
 * Ownership: the library owns contexts, meshes and servers and their device
 * tables; the caller frees them with the matching call.  Host arrays passed
 * in are copied during the call.  Device vectors passed in are caller-owned
 * and must stay alive until the stream work that uses them has finished.
 *
 * Streams: `stream` arguments are hipStream_t values (NULL = the null
 * stream).  Calls taking a stream are asynchronous unless stated otherwise.
 */
#ifndef STDG_H
#define STDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STDG_OK = 0,
  STDG_E_ARG = -1,           /* invalid argument (null, size, range)           */
  STDG_E_UNSUPPORTED = -2,   /* valid but not implemented (e.g. D_h with hanging faces) */
  STDG_E_NOMEM = -3,         /* device or host allocation failed                */
  STDG_E_DEVICE = -4,        /* HIP runtime error or missing GPU                */
  STDG_E_NOT_CONVERGED = -5, /* solver hit its iteration limit (info is filled) */
  STDG_E_NOT_READY = -6,     /* serving ticket not finished yet                 */
  STDG_E_CAPACITY = -7,      /* request larger than the HBM budget              */
  STDG_E_CANCELLED = -8      /* serving request dropped while the server stopped */
} stdg_status;

typedef enum { STDG_FP64 = 0, STDG_FP32 = 1 } stdg_prec;

/* Residual evaluation modes (Section 5, eq. residual; Section 5.4, eq. preconditioner). */
typedef enum {
  STDG_OPERATOR = 0,         /* y = B_h x : x = unknowns (m >= 1), l_0 block taken as 0, no load   */
  STDG_RESIDUAL = 1,         /* y = B_h U - L : U = full trial incl. the l_0 block; L may be NULL  */
  STDG_OPERATOR_PRECOND = 2  /* y = B_h P^{-1} x with P the time-derivative terms (eq. preconditioner) */
} stdg_mode;
/* P is block diagonal: per element and level, the 3x3-per-spatial-mode mass
 * eps|J|DF^{-1}DF^{-T} (mu for H), exact on affine elements and taken at the
 * element centre on trilinear ones.  On axis-aligned meshes P^{-1} is fused
 * into the apply; otherwise the first such call allocates an unknown-sized
 * scratch vector owned by the mesh (STDG_E_NOMEM past the context budget). */

typedef struct stdg_ctx stdg_ctx;
typedef struct stdg_mesh stdg_mesh;
typedef struct stdg_server stdg_server;

/* Library version, (major << 16) | minor. */
int stdg_version(void);

/* Thread-local message of the last failure on this thread ("" if none). */
const char* stdg_last_error(void);

/* sizeof() of each public struct below, so that a binding which mirrors the
 * structs (ctypes, FFI) can check its layout against the built library before
 * passing any of them; 0 for an unknown `which`.  Needs no device. */
enum {
  STDG_STRUCT_MESH_DESC = 0, STDG_STRUCT_MESH_INFO = 1, STDG_STRUCT_SOURCE = 2, STDG_STRUCT_SOLVE_OPTS = 3,
  STDG_STRUCT_SOLVE_INFO = 4, STDG_STRUCT_SERVE_OPTS = 5, STDG_STRUCT_REQUEST = 6, STDG_STRUCT_RESULT = 7,
  STDG_STRUCT_GROUP_INFO = 8
};
size_t stdg_struct_size(int32_t which);

/* Create a context on HIP device `hip_device`.  `hbm_budget_bytes` caps the
 * device memory the context's meshes, solvers and servers may allocate
 * (0 = 90% of the device's free memory).  Fails with STDG_E_DEVICE when no
 * GPU is present. */
int stdg_init(int hip_device, size_t hbm_budget_bytes, stdg_ctx** out);
int stdg_finalize(stdg_ctx* ctx);

/* Mesh and discretisation (Section 2.2-2.3; degrees of eq. spaces:local;
 * elementwise constant eps, mu as in Thm 3.1).  Host arrays, copied. */
typedef struct {
  int64_t n_vertices;
  const double* vertices;   /* [n_vertices][3]                                     */
  int64_t n_elements;
  const int64_t* hexes;     /* [n_elements][8] vertex ids, order above            */
  const int32_t* p;         /* [n_elements] spatial degree, 1 <= p <= 8           */
  const int32_t* q;         /* [n_elements] temporal degree, 1 <= q <= 6          */
  const double* eps;        /* [n_elements] permittivity > 0                      */
  const double* mu;         /* [n_elements] permeability > 0                      */
  const int32_t* nsub;      /* [n_elements] temporal sub-intervals: 1, 2, 4 or 8
                               (n q <= 24), or NULL for one per element          */
} stdg_mesh_desc;

typedef struct {
  int64_t n_elements, n_vertices;
  int64_t n_interior_faces, n_boundary_faces;
  int64_t trial_size, unknown_size, state_size;  /* scalars in each layout      */
  int32_t n_groups;          /* (p, q, affine) kernel groups                     */
  int32_t n_affine, n_nonaffine, n_diagonal_mass;
  int32_t p_max, q_max;
  int64_t device_bytes;      /* device memory held by the mesh                  */
  int32_t work_order;        /* element order of the kernels' work lists: 0 =
                                Morton, T >= 2 = columns of T x T elements      */
} stdg_mesh_info_t;

/* Build faces and neighbours (matching sorted vertex ids), find how each
 * neighbour meets the face (its local face and the symmetry of the square
 * between the two faces' reference coordinates: any hex orientation is
 * accepted; STDG_E_ARG if the shared vertices do not match as a
 * quadrilateral), classify elements as affine (parallelepiped) or trilinear,
 * group them by (p, q, affine), compute offsets and copy everything to the
 * device.  Faces on exactly one element are PEC boundary faces, except 2:1
 * hanging faces (Section 5.2 sums a face's flux terms over the neighbours
 * sharing parts of it): a face whose four quarters are whole faces of four
 * other elements, with mesh vertices at the corners, edge midpoints and
 * centre of its bilinear map (any orientation of the smaller elements, any
 * p and q on either side).  These couple through the centred flux, the
 * neighbours' traces projected onto each side's face modes by half-interval
 * Legendre restrictions, exact for affine faces.  A face split among smaller
 * elements in any other way (found by their centroids at its quarter points)
 * is refused with STDG_E_UNSUPPORTED.  Meshes with hanging faces do not take
 * D_h (stdg_mesh_set_dissipation) and run their serving cycles alone.
 *
 * Local time steps (Section 2.2: each macro-element's slab interval bisected
 * in time; trial space continuous piecewise P_q, test space piecewise
 * P_{q-1}, eq. spaces:local:patch): an element with n = nsub[e] > 1 equal
 * sub-intervals holds 1 + n q trial levels and n q test levels per field and
 * component.  Trial level 0 is the value at the slab start and level 1 the
 * value at the slab end (as with n = 1, so slab transfer, the initial guess
 * and stdg_energy are unchanged); sub-interval j then owns levels
 * 2 + j q .. 1 + (j + 1) q: its interior functions l_2..l_q and, for
 * j < n - 1, the value at its right end.  Test level j q + i is L_i on
 * sub-interval j (L_i(n s - j), s the unit slab coordinate).  Neighbours
 * couple through S_h (Section 4.1, eq. bilinearform:S): the test function
 * projected onto their common temporal test space, piecewise P_{min(q,q')-1}
 * on the coarser of the two partitions.  Such elements and their face
 * neighbours must be affine, and the mesh may not have hanging faces
 * (STDG_E_UNSUPPORTED); batched applies refuse meshes with local time steps
 * (serving requests with them run their cycles alone), and D_h takes them
 * up to p = 4 with q >= 5 (any p below q = 5) within its LDS limit.
 * stdg_load_assemble integrates the source
 * per sub-interval, and the dual norms (stdg_residual_dual_norm, inexact
 * solves) take the test functions of a sub-interval on dt / n. */
int stdg_mesh_upload(stdg_ctx* ctx, const stdg_mesh_desc* desc, stdg_mesh** out);
int stdg_mesh_info(const stdg_mesh* mesh, stdg_mesh_info_t* out);
/* Host copies of the element offsets (n_elements + 1 entries each, any may be NULL). */
int stdg_mesh_offsets(const stdg_mesh* mesh, int64_t* trial_off, int64_t* unknown_off,
                      int64_t* state_off);
int stdg_mesh_free(stdg_mesh* mesh);

/* Order in which the residual kernels visit the elements of each (p, q,
 * affine) group: 0 = Morton order of the centroids; T in 2..64 = columns of
 * T x T elements swept along the third axis (neighbour blocks stay in L2).
 * The upload picks columns of 8 for single-group meshes with small element
 * blocks, else Morton.  Results do not depend on the order (each output reads
 * only its element and its face neighbours).  STDG_E_ARG for other values.
 * Synchronous (host to device copy of the lists); not to be called while work
 * on the mesh is in flight. */
int stdg_mesh_set_order(stdg_mesh* mesh, int32_t order);
/* Autotuner: time `reps` preconditioned operator applies (precision prec,
 * scratch vectors allocated and freed inside the call) for each candidate
 * order (Morton, columns of 4, 8, 16) and keep the fastest (returned in
 * *order_out); then, in that order, time each affine kernel group in each
 * launch variant of stdg_mesh_set_launch and keep the fastest per group
 * (stdg_mesh_group reports it; trilinear groups are timed in the operator
 * mode, which their preconditioned applies run after the P^{-1} pre-pass).
 * Synchronises `stream`; not to be called
 * while other work on the mesh is in flight.  Callers that cache the choices
 * (the Python binding keys a JSON file on the mesh's shape) apply them later
 * with stdg_mesh_set_order and stdg_mesh_set_launch. */
int stdg_mesh_autotune(stdg_mesh* mesh, int prec, double dt, int32_t reps, int32_t* order_out, void* stream);

/* Kernel groups: the elements of one (p, q, affine) triple run through one
 * residual kernel instantiation, one workgroup per element.
 * stdg_mesh_group describes group 0 <= group < n_groups; stdg_mesh_set_launch
 * picks the launch variant of its operator-mode kernels (group = -1: every
 * group).  Affine groups (without D_h; with D_h they keep variant 0):
 *   0  the element's outputs staged through LDS and written as contiguous
 *      8-byte stores (whole cache lines), neighbour faces loaded 3 at a time;
 *   1  outputs written per spatial position, neighbour faces 3 at a time;
 *   2  outputs staged as in 0, neighbour faces loaded one at a time (fewer
 *      registers, more resident waves).
 * Trilinear groups (variant 2, and variant 1 for q = 1 or q > 4, are taken
 * as 0):
 *   0  one workgroup per element;
 *   1  one workgroup per element and test level (q times the workgroups,
 *      each with one level's quadrature mass: for small groups of high
 *      degree).
 * Results are bitwise the same in every variant.  STDG_E_ARG for an unknown
 * group or variant.  Not to be called while work on the mesh is in flight. */
typedef struct {
  int32_t p, q, affine, variant;
  int64_t n_elements;
} stdg_group_info_t;
int stdg_mesh_group(const stdg_mesh* mesh, int32_t group, stdg_group_info_t* out);
int stdg_mesh_set_launch(stdg_mesh* mesh, int32_t group, int32_t variant);

/* Dissipative upwind-type stabilisation D_h (the remark closing Section 4):
 * from this call on, every residual apply and slab solve on `mesh` uses
 * B_h + D_h with
 *   D_h(U, V) = sum_{interior f} (alpha_E [E]_T, [pi v]_T)_f + (alpha_H [H]_T, [pi w]_T)_f
 *             + sum_{PEC f} (alpha_E [E]_T, [v]_T)_f,
 *   alpha_E = c / {sqrt(mu/eps)}, alpha_H = c / {sqrt(eps/mu)}  ({.}: mean of the
 *   two sides, the element's own value on PEC faces; g = 0),
 * pi the temporal projection onto the common test space of the two elements
 * (the same truncation as S_h).  The energy then drops by the dissipation of
 * the slab instead of being conserved.  c = 0 switches it off (the device
 * coefficients are freed).  On affine elements the face metric is constant
 * and the residual kernels carry D_h; on trilinear elements a separate kernel
 * adds it, integrating the face terms with max(a, a') + 2 Gauss points per
 * direction (a, a' = p + 1 of the two sides; a + 2 on PEC faces) and the face
 * metric of the trilinear map at each point.  STDG_E_ARG for c < 0 or
 * non-finite.  Synchronous (host to device copy of 288 bytes per element: the
 * coefficients in FP64 and FP32); not to be called while work on the mesh is
 * in flight. */
int stdg_mesh_set_dissipation(stdg_mesh* mesh, double c);

/* The hot path: the matrix-free space-time residual of one slab (Section 5,
 * eq. residual; evaluation of Section 5.2: mass, curl and flux terms).
 * Affine elements use their constant metric; trilinear elements integrate the
 * mass term with the tensor Gauss-Legendre rule of p + 2 points per direction
 * (Section 5.2, non-affine mass), curl and flux being geometry-free for
 * covariant maps on conforming faces.
 *   dt    slab length (> 0)
 *   prec  STDG_FP64 (double vectors) or STDG_FP32 (float vectors, FP32 accumulation)
 *   mode  stdg_mode above; x_dev layout = unknowns (OPERATOR*) or full trial (RESIDUAL)
 *   load_dev  residual-layout load vector L (RESIDUAL mode only; NULL = 0)
 *   y_dev residual layout, overwritten.  x_dev and y_dev must not overlap.
 * Device pointers; asynchronous on `stream`. */
int stdg_residual_apply(const stdg_mesh* mesh, double dt, int prec, int mode,
                        const void* x_dev, const void* load_dev, void* y_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as stdg_residual_apply, same arguments and results, that
 * allocates nothing.  Preconditioned applies on meshes with a non-diagonal
 * metric (sheared or trilinear elements) scale the input by P^{-1} into a
 * static device array of stdg_noalloc_scratch_bytes() bytes (64 MiB; each
 * device holds its own copy until the process ends) instead of the mesh's
 * scratch: STDG_E_CAPACITY when unknown_size * (4 or 8) exceeds it.  Meshes
 * with several kernel groups launch the groups one after another on
 * `stream` (no side streams).  Every call on a device shares that device's
 * array, which keeps the last call's contents (each call overwrites what it
 * reads): calls that overlap on one device, on different streams or threads,
 * race and give wrong results.  Device pointers; asynchronous on `stream`. */
int stdg_residual_apply_noalloc(const stdg_mesh* mesh, double dt, int prec, int mode,
                                const void* x_dev, const void* load_dev, void* y_dev, void* stream);
size_t stdg_noalloc_scratch_bytes(void);

/* Measurement utility, no operation of the method: copies `bytes` bytes from
 * src to dst (device pointers, both 16-byte aligned, bytes a multiple of 16,
 * no overlap) with the library's streaming kernel - 16-byte non-temporal
 * loads and stores, grid-stride, 32 blocks per compute unit - so that
 * 2 * bytes cross HBM.  Its rate is the practical bandwidth ceiling the
 * memory-bound kernels are compared with, and its traffic counters calibrate
 * theirs.  Asynchronous on `stream`.  STDG_E_ARG for NULL, misaligned or
 * overlapping buffers; bytes = 0 does nothing. */
int stdg_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Current density of the load L(V) = (J, v) (eq. bilinearform:C):
 * kind 0 = none; kind 1 = J(x,t) = dir * amp * exp(-|x - center|^2 / (2 sigma_x^2))
 *                          * sin(2 pi f0 (t - t0)) * exp(-(t - t0)^2 / (2 sigma_t^2)). */
typedef struct {
  int32_t kind;
  double amp;
  double center[3];
  double sigma_x, f0, t0, sigma_t;
  double dir[3];
} stdg_source;

/* L_E[c,i,s] = int_{I_n} int_K J . (DF^{-T} e_c phi_s) L_i dx dt by tensor Gauss
 * quadrature (p + 3 points per space direction, q + 3 in time); L_H = 0 (g = 0).
 * Writes the residual-layout FP64 vector load_dev for the slab (t0, t0 + dt]. */
int stdg_load_assemble(const stdg_mesh* mesh, const stdg_source* src, double t0, double dt,
                       double* load_dev, void* stream);

/* Cavity-mode superposition initial field on the unit cube,
 * E = sum_r (A_r cos(m pi x) sin(n pi y) sin(l pi z), B_r sin cos sin, C_r sin sin cos), H = 0,
 * L2-projected onto the covariant discrete space: state_dev (FP64 state layout).
 * Affine elements only. */
int stdg_project_modes(const stdg_mesh* mesh, int32_t n_modes, const int32_t* mnl,
                       const double* abc, double* state_dev, void* stream);

/* Slab solve (Section 3 eq. weakform / Section 4 eq. weakform_stabilized) by
 * right-preconditioned restarted GMRES (Section 5.4, eq. preconditioner). */
typedef struct {
  int32_t inner_prec;  /* STDG_FP64: plain FP64 GMRES; STDG_FP32: FP32 operator inside
                          FP64 iterative refinement                              */
  int32_t restart;     /* GMRES restart length (default 10, at most 15)          */
  int32_t max_iters;   /* total inner iterations allowed (default 500)           */
  int32_t max_refine;  /* FP64 residual re-evaluations allowed with FP32 inner    
                          applies (one per restart cycle; default 100)           */
  double rtol;         /* stop when ||L - B U||_2 <= rtol ||L - B U_0||_2 (FP64)  */
  double inner_rtol;   /* relative tolerance of each inner GMRES (FP32 inner)    */
  int32_t krylov_prec; /* storage of the Krylov basis: STDG_FP64 (default), or
                          STDG_FP32 with FP32 inner applies (sums stay FP64)     */
  double eta_tol;      /* inexact solve (Section 5.3): > 0 also stops once this
                          slab's term of the iteration-error bound eta_it^2
                          (eq. a_posteriori:iteration) is <= eta_tol^2; 0 = off  */
  double eta_t_final;  /* t_N of that bound (final time, slabs from t = 0), > 0
                          when eta_tol > 0                                       */
  int32_t use_graph;   /* 1: replay each restart cycle (start vector, up to
                          `restart` Arnoldi iterations of apply and two basis
                          passes, least-squares update of the iterate) as one
                          captured HIP graph, kept with the mesh's solver
                          (captured at the second cycle, recaptured when dt or
                          the mesh's launch set-up changes); results are bitwise
                          those of the direct launches.  0 = direct launches.
                          Either way the host waits once per restart cycle.    */
} stdg_solve_opts;

typedef struct {
  int32_t iters;        /* inner GMRES iterations (operator applications)        */
  int32_t refinements;  /* outer FP64 residual evaluations                      */
  double rel_res;       /* final ||L - B U|| / ||L - B U_0|| in FP64             */
  double energy_start;  /* discrete energy (eq. stability:energydef) at t0      */
  double energy_end;    /* ... at t0 + dt                                       */
  double eta2;          /* with eta_tol: this slab's term of eta_it^2 at the final
                           iterate (sum the terms over slabs for eta_it^2)       */
} stdg_solve_info;

/* state_dev (FP64 state layout) holds the fields at t0 on entry and at t0 + dt
 * on return (the l_1 block, i.e. continuity in time between slabs).
 * load_dev: residual-layout FP64 load of this slab, or NULL (J = 0).
 * slab_U_dev: optional FP64 full-trial output of the slab solution (NULL = none).
 * Synchronises `stream`.  STDG_E_NOT_CONVERGED still fills *info and state.
 * The solver's device memory (Krylov basis and work vectors, counted against
 * the context budget) is allocated on the first call and kept on the mesh for
 * the next ones (a march of slabs allocates once); it is reallocated when the
 * precisions or the restart length change and freed by stdg_mesh_free.  A call
 * made while another thread solves on the same mesh uses memory of its own. */
int stdg_slab_solve(const stdg_mesh* mesh, double t0, double dt, const double* load_dev,
                    const stdg_solve_opts* opts, double* state_dev, double* slab_U_dev,
                    stdg_solve_info* info, void* stream);

/* Dual norms of a residual-layout FP64 vector r (e.g. from STDG_RESIDUAL) in
 * W_h' with the L2(I_n; L2(Omega)) norm (Section 5.3: the Riesz representor is
 * an L2 projection): norms_out[0] = ||r_E||^2, norms_out[1] = ||r_H||^2.
 * Exact on every element: affine elements invert their constant metric,
 * trilinear ones solve with their quadrature mass (the residual's (p+2)-point
 * rule) by preconditioned conjugate gradients to 1e-14.  Synchronises `stream`. */
int stdg_residual_dual_norm(const stdg_mesh* mesh, double dt, const double* r_dev, double* norms_out,
                            void* stream);

/* Discrete energy 1/2 int (eps E.E + mu H.H) of an FP64 state (eq. stability:energydef);
 * on trilinear elements with the mass rule of the residual (p + 2 Gauss points per direction). */
int stdg_energy(const stdg_mesh* mesh, const double* state_dev, double* energy_out, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: independent PEC cavity solves (a mesh, an initial field, a current
 * and a number of slabs each), marched slab by slab (Section 2.2, time slabs;
 * each slab solved as stdg_slab_solve does) by one server thread per server.
 *
 * Admission: a request is admitted when a contiguous reservation of its
 * device footprint (mesh tables, state, load, Krylov vectors; reported in
 * stdg_result.device_bytes) fits in the server's HBM arena and fewer than
 * max_active requests are in flight; otherwise it waits in FIFO order.
 * Admitted requests run concurrently, each on its own stream: the server
 * advances whichever request's last step has completed (one GMRES iteration,
 * restart cycle or slab boundary at a time), so requests that arrive while
 * others run join at the next step and their work overlaps on the device.
 * Each request's arithmetic is independent of the others (own buffers, fixed
 * reduction order): its result is bitwise the same alone and in a mix.
 * ------------------------------------------------------------------------- */
typedef struct {
  size_t hbm_budget;     /* bytes of the server's device arena (0 = 16 GiB)        */
  int32_t max_active;    /* requests in flight at once (0 = 16)                    */
  int32_t inner_prec;    /* stdg_solve_opts fields, applied to every slab          */
  int32_t restart;
  int32_t max_iters;     /* per slab */
  int32_t max_refine;
  double rtol;
  double inner_rtol;
  int32_t krylov_prec;
  double eta_rel;        /* > 0: inexact solves (Section 5.3): each request stops a
                            slab once its term of eta_it^2 (t_N = n_slabs dt) is
                            <= (eta_rel sqrt(2 E(t0)))^2 / n_slabs, so that
                            eta_it <= eta_rel sqrt(2 E(t0)) over the request;
                            0 = solve every slab to rtol                         */
  int32_t use_graph;     /* as stdg_solve_opts.use_graph, for every request      */
  int32_t batch_cycles;  /* 1: requests whose meshes are one affine kernel group
                            of the same (p, q) with a diagonal metric and no D_h
                            (FP32 inner applies) run their restart cycles
                            together: one launch per apply and per basis pass
                            for up to 16 requests, each on its own segment of
                            the grid with its own block partition, so results
                            are bitwise those of the request alone; a pending
                            cycle waits at most 0.5 ms for partners.  0: every
                            request alone                                     */
} stdg_serve_opts;

typedef struct {
  stdg_mesh_desc mesh;       /* host arrays, copied by stdg_serve_submit            */
  double t0, dt;             /* start time and slab length (> 0)                    */
  int32_t n_slabs;           /* >= 1                                                */
  stdg_source source;        /* current density (kind 0 = none), load per slab      */
  int32_t n_modes;           /* initial field: cavity-mode superposition, as        */
  const int32_t* mnl;        /*   stdg_project_modes (affine meshes), or            */
  const double* abc;
  const double* init_state;  /*   an FP64 state (host, state layout) if not NULL    */
  double c_diss;             /* >= 0: dissipative stabilisation D_h with this c, as  */
                             /*   stdg_mesh_set_dissipation (0 = off)                */
  int64_t init_state_size;   /* entries at init_state: must equal the mesh's state
                                size (sum of 6 (p+1)^3), else STDG_E_ARG; ignored
                                when init_state is NULL                             */
} stdg_request;

typedef struct {
  int32_t status;            /* STDG_OK, STDG_E_NOT_CONVERGED (a slab missed rtol),
                                STDG_E_CANCELLED, or the error that stopped it      */
  int32_t slabs_done;
  int64_t iters;             /* inner GMRES iterations over all slabs               */
  double max_rel_res;        /* largest final relative residual over the slabs      */
  double energy_start;       /* discrete energy at t0                               */
  double energy_end;         /* ... at the end of the last slab done                */
  double t_submit, t_admit, t_done;  /* seconds on the server clock                 */
  int64_t state_size;        /* entries of the final state                          */
  int64_t device_bytes;      /* reservation the request held                        */
  double eta_it;             /* with eta_rel: the accumulated iteration-error bound */
  double* state;             /* in: caller host buffer for the final state, or NULL */
  int64_t state_capacity;    /* in: entries available at state                      */
  int64_t batched_cycles;    /* restart cycles run together with other requests     */
} stdg_result;

/* Start a server on the context's device.  The server thread owns the
 * context's device while it runs: do not use the same context from other
 * threads until stdg_serve_stop returns. */
int stdg_serve_start(stdg_ctx* ctx, const stdg_serve_opts* opts, stdg_server** out);
/* Queue a request (thread-safe; every array is copied before return).  The
 * mesh is validated and analysed during the call (faces, metric, kernel
 * groups), so mesh errors are returned here (STDG_E_ARG, STDG_E_UNSUPPORTED);
 * STDG_E_CAPACITY if the request's footprint exceeds the whole arena.  The
 * request's latency clock (t_submit) starts on entry. */
int stdg_serve_submit(stdg_server* server, const stdg_request* req, uint64_t* ticket);
/* STDG_E_NOT_READY until the request has finished; then fills *out (copying
 * the final state into out->state when out->state_capacity suffices, else
 * STDG_E_ARG and the result is kept) and releases the ticket.  Thread-safe. */
int stdg_serve_poll(stdg_server* server, uint64_t ticket, stdg_result* out);
/* Seconds on the server clock (the clock of t_submit, t_admit, t_done). */
double stdg_serve_clock(const stdg_server* server);
/* Stop: waits for the device work in flight, drops requests still queued or
 * running and results not yet polled, frees the arena; the handle is invalid
 * afterwards. */
int stdg_serve_stop(stdg_server* server);

#ifdef __cplusplus
}
#endif

#endif /* STDG_H */
