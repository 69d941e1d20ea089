// Once-per-slab kernels around the residual: the load L(V) = (J, v)
// (eq. bilinearform:C), the L2 projection of cavity-mode initial fields, and
// the discrete energy 1/2 int (eps E.E + mu H.H) (eq. stability:energydef),
// all in FP64.
#include <cmath>

#include "internal.h"

namespace stdg {

namespace {

// n-point Gauss-Legendre rule on [0, 1] (n <= 16) by Newton iteration on P_n.
__host__ __device__ void gauss01(int n, double* xs, double* ws) {
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double pn = 0.0, pm = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      pn = p1;
      pm = n == 1 ? 1.0 : p0;
      double dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    pn = p1;
    pm = n == 1 ? 1.0 : p0;
    double dp = n * (z * pn - pm) / (z * z - 1.0);
    xs[i] = 0.5 * (1.0 - z);
    ws[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
}

struct LoadParams {
  const ElemInfo* info;
  const double* verts;
  double* out;
  stdg_source src;
  double t0, dt;
};

__device__ double leg(int j, double xi) {
  // orthonormal Legendre on [0,1] by Bonnet's recurrence
  double u = 2.0 * xi - 1.0, p0 = 1.0, p1 = u;
  if (j == 0) return 1.0;
  for (int k = 1; k < j; ++k) {
    double p2 = ((2.0 * k + 1.0) * u * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return sqrt(2.0 * j + 1.0) * p1;
}

__device__ void trilinear(const double* X, double x, double y, double z, double F[3], double DF[3][3]) {
  for (int c = 0; c < 3; ++c) {
    F[c] = 0.0;
    DF[c][0] = DF[c][1] = DF[c][2] = 0.0;
  }
  for (int v = 0; v < 8; ++v) {
    const int b0 = v & 1, b1 = (v >> 1) & 1, b2 = (v >> 2) & 1;
    const double fx = b0 ? x : 1.0 - x, fy = b1 ? y : 1.0 - y, fz = b2 ? z : 1.0 - z;
    const double sx = b0 ? 1.0 : -1.0, sy = b1 ? 1.0 : -1.0, sz = b2 ? 1.0 : -1.0;
    const double N = fx * fy * fz;
    const double d0 = sx * fy * fz, d1 = fx * sy * fz, d2 = fx * fy * sz;
    for (int c = 0; c < 3; ++c) {
      const double Xc = X[3 * v + c];
      F[c] += N * Xc;
      DF[c][0] += d0 * Xc;
      DF[c][1] += d1 * Xc;
      DF[c][2] += d2 * Xc;
    }
  }
}

__device__ double inv3(const double A[3][3], double B[3][3]) {
  double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
               A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  double id = 1.0 / det;
  B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) * id;
  B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
  B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
  B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) * id;
  B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
  B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
  B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) * id;
  B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
  B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
  return det;
}


// Space-time separable current J(x, t) = dir amp g(x) h(t) (stdg_source kind 1):
//   L_E[c, i, s] = T_i S_c(s),  T_i = dt sum_t w_t L_i(tau_t) h(t0 + tau_t dt),
// (with n sub-intervals, test level j q + i: (dt / n) sum_t w_t L_i(tau_t)
// h(t0 + (j + tau_t) dt / n), the rule applied per sub-interval),
//   S_c(s) = amp sum_g w_g phi_s(x_g) g(F(x_g)) |J| (DF^{-1} dir)_c,
// with Gauss rules of q + 3 points in time and p + 3 per space direction; S is
// sum factorised like the projection (point values in shared memory, then one
// direction at a time).  Dynamic shared memory: 3 nx^3 + nx^2 a + nx a^2
// doubles, nx = a + 2.
__global__ void load_kernel(LoadParams P) {
  extern __shared__ double sh[];
  __shared__ double qx[kMaxA + 2], qw[kMaxA + 2], Bt[(kMaxA + 2) * kMaxA], tx[kMaxQ + 3], tw[kMaxQ + 3],
      Ti[kMaxLocalLevels];
  const int e = blockIdx.x;
  const ElemInfo I = P.info[e];
  const int a = I.a, q = I.q, a2 = a * a, a3 = a2 * a;
  const int ns = I.nsub, nl = q * ns;  // sub-intervals, test levels
  double* out = P.out + I.unk_off;
  if (P.src.kind != 1) {
    for (int idx = threadIdx.x; idx < 6 * nl * a3; idx += blockDim.x) out[idx] = 0.0;
    return;
  }
  const int nx = a + 2, nx2 = nx * nx, nx3 = nx2 * nx, nt = q + 3;
  if (threadIdx.x == 0) {
    gauss01(nx, qx, qw);
    gauss01(nt, tx, tw);
  }
  __syncthreads();
  const stdg_source& S = P.src;
  if ((int)threadIdx.x < nl) {
    const int j = (int)threadIdx.x / q, i = (int)threadIdx.x - j * q;
    const double hs = P.dt / ns;
    double v = 0.0;
    for (int g = 0; g < nt; ++g) {
      const double tt = P.t0 + (j + tx[g]) * hs - S.t0;
      const double h = sin(2.0 * M_PI * S.f0 * tt) * exp(-tt * tt / (2.0 * S.sigma_t * S.sigma_t));
      v += tw[g] * leg(i, tx[g]) * h;
    }
    Ti[threadIdx.x] = hs * v;
  }
  for (int k = threadIdx.x; k < nx * a; k += blockDim.x) {
    const int g = k / a, j = k - g * a;
    Bt[k] = qw[g] * leg(j, qx[g]);
  }
  const double* X = P.verts + 24 * e;
  double* F = sh;
  double* T1 = sh + 3 * nx3;
  double* T2 = T1 + nx2 * a;
  for (int pt = threadIdx.x; pt < nx3; pt += blockDim.x) {
    const int g1 = pt % nx, g2 = (pt / nx) % nx, g3 = pt / nx2;
    double xp[3], DF[3][3], Di[3][3];
    trilinear(X, qx[g1], qx[g2], qx[g3], xp, DF);
    const double det = inv3(DF, Di);
    const double dx = xp[0] - S.center[0], dy = xp[1] - S.center[1], dz = xp[2] - S.center[2];
    const double gsp = S.amp * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * S.sigma_x * S.sigma_x)) * det;
    // J . DF^{-T} e_c = (DF^{-1} J)_c
    for (int c = 0; c < 3; ++c)
      F[c * nx3 + pt] = gsp * (Di[c][0] * S.dir[0] + Di[c][1] * S.dir[1] + Di[c][2] * S.dir[2]);
  }
  __syncthreads();
  for (int c = 0; c < 3; ++c) {
    const double* Fc = F + c * nx3;
    for (int o = threadIdx.x; o < nx2 * a; o += blockDim.x) {  // [g3][g2][j]
      const int j = o % a, g23 = o / a;
      double acc = 0.0;
      for (int g1 = 0; g1 < nx; ++g1) acc += Bt[g1 * a + j] * Fc[g23 * nx + g1];
      T1[o] = acc;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < nx * a2; o += blockDim.x) {  // [g3][k][j]
      const int j = o % a, k = (o / a) % a, g3 = o / a2;
      double acc = 0.0;
      for (int g2 = 0; g2 < nx; ++g2) acc += Bt[g2 * a + k] * T1[(g3 * nx + g2) * a + j];
      T2[o] = acc;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < a3; s += blockDim.x) {  // [l][k][j]
      const int jk = s % a2, l = s / a2;
      double acc = 0.0;
      for (int g3 = 0; g3 < nx; ++g3) acc += Bt[g3 * a + l] * T2[g3 * a2 + jk];
      for (int i = 0; i < nl; ++i) {
        out[((int64_t)c * nl + i) * a3 + s] = Ti[i] * acc;      // E part
        out[((int64_t)(3 + c) * nl + i) * a3 + s] = 0.0;        // H part: g = 0
      }
    }
    __syncthreads();
  }
}

struct ProjParams {
  const ElemInfo* info;
  const ElemMetric* metric;
  const int64_t* state_off;
  const double* verts;
  double* out;
  int n_modes;
  const int32_t* mnl;
  const double* abc;
};

// L2 projection on affine elements, sum factorised over the tensor Gauss rule
// of a + 3 points per direction: the field is evaluated once per point (mapped
// covariantly, times |J|) into shared memory, contracted one direction at a
// time against w_g L_j(x_g), and the per-mode 3x3 mass G = |J| DF^{-1} DF^{-T}
// is inverted at the end (the mass of an affine element is G (x) I).
// Dynamic shared memory: 3 nx^3 + nx^2 a + nx a^2 doubles, nx = a + 3.
__global__ void project_kernel(ProjParams P) {
  extern __shared__ double sh[];
  __shared__ double qx[kMaxA + 3], qw[kMaxA + 3], Bt[(kMaxA + 3) * kMaxA];
  const int e = blockIdx.x;
  const ElemInfo I = P.info[e];
  const int a = I.a, a2 = a * a, a3 = a2 * a;
  const int nx = a + 3, nx2 = nx * nx, nx3 = nx2 * nx;
  if (threadIdx.x == 0) gauss01(nx, qx, qw);
  __syncthreads();
  for (int k = threadIdx.x; k < nx * a; k += blockDim.x) {
    const int g = k / a, j = k - g * a;
    Bt[k] = qw[g] * leg(j, qx[g]);
  }
  const double* X = P.verts + 24 * e;
  double F0[3], DF[3][3], Di[3][3];
  trilinear(X, 0.5, 0.5, 0.5, F0, DF);
  const double det = inv3(DF, Di);
  double* F = sh;
  double* T1 = sh + 3 * nx3;
  double* T2 = T1 + nx2 * a;
  for (int pt = threadIdx.x; pt < nx3; pt += blockDim.x) {
    const int g1 = pt % nx, g2 = (pt / nx) % nx, g3 = pt / nx2;
    double xp[3], DFp[3][3];
    trilinear(X, qx[g1], qx[g2], qx[g3], xp, DFp);
    double E[3] = {0.0, 0.0, 0.0};
    for (int r = 0; r < P.n_modes; ++r) {
      const double kx = M_PI * P.mnl[3 * r] * xp[0], ky = M_PI * P.mnl[3 * r + 1] * xp[1],
                   kz = M_PI * P.mnl[3 * r + 2] * xp[2];
      const double sx = sin(kx), cx = cos(kx), sy = sin(ky), cy = cos(ky), sz = sin(kz), cz = cos(kz);
      E[0] += P.abc[3 * r] * cx * sy * sz;
      E[1] += P.abc[3 * r + 1] * sx * cy * sz;
      E[2] += P.abc[3 * r + 2] * sx * sy * cz;
    }
    // E . DF^{-T} e_c |J| = (DF^{-1} E)_c |J|
    for (int c = 0; c < 3; ++c) F[c * nx3 + pt] = det * (Di[c][0] * E[0] + Di[c][1] * E[1] + Di[c][2] * E[2]);
  }
  __syncthreads();
  double* out = P.out + P.state_off[e];
  for (int c = 0; c < 3; ++c) {
    const double* Fc = F + c * nx3;
    for (int o = threadIdx.x; o < nx2 * a; o += blockDim.x) {  // [g3][g2][j]
      const int j = o % a, g23 = o / a;
      double acc = 0.0;
      for (int g1 = 0; g1 < nx; ++g1) acc += Bt[g1 * a + j] * Fc[g23 * nx + g1];
      T1[o] = acc;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < nx * a2; o += blockDim.x) {  // [g3][k][j]
      const int j = o % a, k = (o / a) % a, g3 = o / a2;
      double acc = 0.0;
      for (int g2 = 0; g2 < nx; ++g2) acc += Bt[g2 * a + k] * T1[(g3 * nx + g2) * a + j];
      T2[o] = acc;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < a3; s += blockDim.x) {  // [l][k][j]
      const int jk = s % a2, l = s / a2;
      double acc = 0.0;
      for (int g3 = 0; g3 < nx; ++g3) acc += Bt[g3 * a + l] * T2[g3 * a2 + jk];
      out[(int64_t)c * a3 + s] = acc;
    }
    __syncthreads();
  }
  // c_s = G^{-1} b_s with G = |J| DF^{-1} DF^{-T}
  double G[3][3], Gi[3][3];
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) G[c][d] = det * (Di[c][0] * Di[d][0] + Di[c][1] * Di[d][1] + Di[c][2] * Di[d][2]);
  inv3(G, Gi);
  for (int s = threadIdx.x; s < a3; s += blockDim.x) {
    const double b0 = out[s], b1 = out[a3 + s], b2 = out[2 * a3 + s];
    for (int c = 0; c < 3; ++c) {
      out[(int64_t)c * a3 + s] = Gi[c][0] * b0 + Gi[c][1] * b1 + Gi[c][2] * b2;
      out[(int64_t)(3 + c) * a3 + s] = 0.0;
    }
  }
}

// per-element energy 1/2 (e^T M_eps e + h^T M_mu h): affine elements from the
// constant metric, trilinear ones with the mass rule of the residual (Gauss,
// a + 1 points per direction): 1/2 sum_g w_g (eps E.G E + mu H.G H)(x_g) in
// reference coordinates, G = |J| DF^{-1} DF^{-T}
__global__ void energy_kernel(const ElemInfo* info, const ElemMetric* metric, const double* verts,
                              const int64_t* state_off, int64_t ne, const double* state, double* partial) {
  const int64_t e = blockIdx.x;
  if (e >= ne) return;
  const ElemInfo I = info[e];
  const int a = I.a, a3 = a * a * a;
  const double* m = metric[e].m;
  const double* st = state + state_off[e];
  __shared__ double red[256];
  __shared__ double qx[kMaxA + 1], qw[kMaxA + 1], Bt[(kMaxA + 1) * kMaxA];
  double acc = 0.0;
  if (I.flags & kAffine) {
    for (int s = threadIdx.x; s < a3; s += blockDim.x) {
      for (int f = 0; f < 2; ++f) {
        const double* M = m + 6 * f;
        const double v0 = st[(3 * f + 0) * a3 + s], v1 = st[(3 * f + 1) * a3 + s], v2 = st[(3 * f + 2) * a3 + s];
        acc += M[0] * v0 * v0 + M[1] * v1 * v1 + M[2] * v2 * v2 +
               2.0 * (M[3] * v0 * v1 + M[4] * v0 * v2 + M[5] * v1 * v2);
      }
    }
  } else {
    const int nq = a + 1, nq3 = nq * nq * nq;
    if (threadIdx.x == 0) gauss01(nq, qx, qw);
    __syncthreads();
    for (int k = threadIdx.x; k < nq * a; k += blockDim.x) {
      const int g = k / a, j = k - g * a;
      Bt[k] = sqrt(qw[g]) * leg(j, qx[g]);
    }
    __syncthreads();
    const double kap[2] = {metric[e].eps, metric[e].mu};
    for (int pt = threadIdx.x; pt < nq3; pt += blockDim.x) {
      const int g1 = pt % nq, g2 = (pt / nq) % nq, g3 = pt / (nq * nq);
      double F[3], DF[3][3], Di[3][3];
      trilinear(verts + 24 * e, qx[g1], qx[g2], qx[g3], F, DF);
      const double det = inv3(DF, Di);
      double G[3][3];
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) G[c][d] = det * (Di[c][0] * Di[d][0] + Di[c][1] * Di[d][1] + Di[c][2] * Di[d][2]);
      for (int f = 0; f < 2; ++f) {
        double u[3] = {0.0, 0.0, 0.0};
        for (int l = 0; l < a; ++l)
          for (int k = 0; k < a; ++k) {
            const double bkl = Bt[g3 * a + l] * Bt[g2 * a + k];
            for (int j = 0; j < a; ++j) {
              const double b = bkl * Bt[g1 * a + j];
              const int s = (l * a + k) * a + j;
              for (int c = 0; c < 3; ++c) u[c] += b * st[(3 * f + c) * a3 + s];
            }
          }
        double q = 0.0;
        for (int c = 0; c < 3; ++c)
          for (int d = 0; d < 3; ++d) q += u[c] * G[c][d] * u[d];
        acc += kap[f] * q;
      }
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[e] = 0.5 * red[0];
}

// Riesz representor of a residual-layout vector per element: sum over levels
// and spatial modes of R_f . (G^{-1} R_f) with the unit-coefficient metric
// (exact mass inverse on affine elements; the centre metric on trilinear ones).
// partial[2 e + f] for the fields f = E, H (divided by dt by the caller).
// With n sub-intervals a test function lives on dt / n: the sum times n.
__global__ void dual_norm_kernel(const ElemInfo* info, const ElemMetric* metric, int64_t ne, const double* R,
                                 double* partial) {
  const int64_t e = blockIdx.x;
  if (e >= ne) return;
  const ElemInfo I = info[e];
  if (!(I.flags & kAffine)) return;  // trilinear elements: the exact mass solve of dualnorm.hip
  const int per = I.q * I.nsub * I.a * I.a * I.a;
  const double* mm = metric[e].m;
  const double kap[2] = {metric[e].eps, metric[e].mu};
  __shared__ double red[2][256];
  double acc[2] = {0.0, 0.0};
  for (int idx = threadIdx.x; idx < per; idx += blockDim.x) {
    for (int f = 0; f < 2; ++f) {
      const double* Mi = mm + 12 + 6 * f;
      const double* rb = R + I.unk_off + (int64_t)3 * f * per + idx;
      const double r0 = rb[0], r1 = rb[per], r2 = rb[2 * per];
      acc[f] += kap[f] * (Mi[0] * r0 * r0 + Mi[1] * r1 * r1 + Mi[2] * r2 * r2 +
                          2.0 * (Mi[3] * r0 * r1 + Mi[4] * r0 * r2 + Mi[5] * r1 * r2));
    }
  }
  red[0][threadIdx.x] = acc[0];
  red[1][threadIdx.x] = acc[1];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * e] = red[0][0] * I.nsub;
    partial[2 * e + 1] = red[1][0] * I.nsub;
  }
}

// out[f] = scale * sum_e partial[2 e + f], f = 0, 1, in a fixed order
__global__ void sum2_kernel(const double* v, int64_t n, double scale, double* out) {
  __shared__ double red[2][512];
  double a0 = 0.0, a1 = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    a0 += v[2 * i];
    a1 += v[2 * i + 1];
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = scale * red[0][0];
    out[1] = scale * red[1][0];
  }
}

// fixed-order sum of n values by one block (deterministic)
__global__ void sum_kernel(const double* v, int64_t n, double* out) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += v[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

int energy_async(const Mesh* m, const double* state, double* d_partial, double* d_out, hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3((unsigned)m->ne), dim3(128), 0, s, m->d_info, m->d_metric, m->d_verts,
                     m->d_state_off, m->ne, state, d_partial);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1024), 0, s, d_partial, m->ne, d_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "energy kernels");
  return STDG_OK;
}

int dual_norms_async(const Mesh* m, double dt, const double* R, double* d_partial, double* d_out, hipStream_t s) {
  hipLaunchKernelGGL(dual_norm_kernel, dim3((unsigned)m->ne), dim3(256), 0, s, m->d_info, m->d_metric, m->ne, R,
                     d_partial);
  if (m->n_nonaffine > 0) {
    int rc = launch_dual_norm_trilinear(m, R, d_partial, s);
    if (rc != STDG_OK) return rc;
  }
  hipLaunchKernelGGL(sum2_kernel, dim3(1), dim3(512), 0, s, d_partial, m->ne, 1.0 / dt, d_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "dual norm kernels");
  return STDG_OK;
}

int ensure_state_off(Mesh* m) {
  if (m->d_state_off) return STDG_OK;
  int rc = dev_alloc(m->ctx, (void**)&m->d_state_off, sizeof(int64_t) * (m->ne + 1));
  if (rc != STDG_OK) return rc;
  m->device_bytes += sizeof(int64_t) * (m->ne + 1);
  STDG_HIP(hipMemcpy(m->d_state_off, m->state_off.data(), sizeof(int64_t) * (m->ne + 1), hipMemcpyHostToDevice));
  return STDG_OK;
}

}  // namespace stdg

using namespace stdg;

extern "C" {

int stdg_load_assemble(const stdg_mesh* mesh, const stdg_source* src, double t0, double dt, double* load_dev,
                       void* stream) {
  if (!mesh || !src || !load_dev) return fail(STDG_E_ARG, "stdg_load_assemble: NULL argument");
  if (!(dt > 0.0)) return fail(STDG_E_ARG, "stdg_load_assemble: dt must be > 0");
  if (src->kind != 0 && src->kind != 1) return fail(STDG_E_ARG, "stdg_load_assemble: unknown source kind");
  if (src->kind == 1 && (!(src->sigma_x > 0.0) || !(src->sigma_t > 0.0)))
    return fail(STDG_E_ARG, "stdg_load_assemble: sigma_x and sigma_t must be > 0");
  const Mesh& m = mesh->m;
  LoadParams P;
  P.info = m.d_info;
  P.verts = m.d_verts;
  P.out = load_dev;
  P.src = *src;
  P.t0 = t0;
  P.dt = dt;
  const int amax = m.p_max + 1, nx = amax + 2;
  const size_t shb = sizeof(double) * (3 * nx * nx * nx + nx * nx * amax + nx * amax * amax);
  hipLaunchKernelGGL(load_kernel, dim3((unsigned)m.ne), dim3(256), shb, (hipStream_t)stream, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "load kernel");
  return STDG_OK;
}

int stdg_project_modes(const stdg_mesh* mesh, int32_t n_modes, const int32_t* mnl, const double* abc,
                       double* state_dev, void* stream) {
  if (!mesh || !state_dev || n_modes < 0 || (n_modes > 0 && (!mnl || !abc)))
    return fail(STDG_E_ARG, "stdg_project_modes: invalid argument");
  Mesh& m = const_cast<stdg_mesh*>(mesh)->m;
  if (m.n_nonaffine > 0) return fail(STDG_E_UNSUPPORTED, "stdg_project_modes: affine elements only");
  int rc = ensure_state_off(&m);
  if (rc != STDG_OK) return rc;
  int32_t* d_mnl = nullptr;
  double* d_abc = nullptr;
  size_t nb = sizeof(int32_t) * 3 * (n_modes > 0 ? n_modes : 1), nd = sizeof(double) * 3 * (n_modes > 0 ? n_modes : 1);
  if ((rc = dev_alloc(m.ctx, (void**)&d_mnl, nb)) != STDG_OK) return rc;
  if ((rc = dev_alloc(m.ctx, (void**)&d_abc, nd)) != STDG_OK) {
    dev_free(m.ctx, d_mnl, nb);
    return rc;
  }
  if (n_modes > 0) {
    STDG_HIP(hipMemcpy(d_mnl, mnl, sizeof(int32_t) * 3 * n_modes, hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(d_abc, abc, sizeof(double) * 3 * n_modes, hipMemcpyHostToDevice));
  }
  ProjParams P;
  P.info = m.d_info;
  P.metric = m.d_metric;
  P.state_off = m.d_state_off;
  P.verts = m.d_verts;
  P.out = state_dev;
  P.n_modes = n_modes;
  P.mnl = d_mnl;
  P.abc = d_abc;
  const int amax = m.p_max + 1, nx = amax + 3;
  const size_t shb = sizeof(double) * (3 * nx * nx * nx + nx * nx * amax + nx * amax * amax);
  hipLaunchKernelGGL(project_kernel, dim3((unsigned)m.ne), dim3(256), shb, (hipStream_t)stream, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "project kernel");
  STDG_HIP(hipStreamSynchronize((hipStream_t)stream));
  dev_free(m.ctx, d_mnl, nb);
  dev_free(m.ctx, d_abc, nd);
  return STDG_OK;
}

int stdg_residual_dual_norm(const stdg_mesh* mesh, double dt, const double* r_dev, double* norms_out,
                            void* stream) {
  if (!mesh || !r_dev || !norms_out) return fail(STDG_E_ARG, "stdg_residual_dual_norm: NULL argument");
  if (!(dt > 0.0)) return fail(STDG_E_ARG, "stdg_residual_dual_norm: dt must be > 0");
  Mesh& m = const_cast<stdg_mesh*>(mesh)->m;
  double* d_tmp = nullptr;
  const size_t nb = sizeof(double) * (2 * m.ne + 2);
  int rc;
  if ((rc = dev_alloc(m.ctx, (void**)&d_tmp, nb)) != STDG_OK) return rc;
  rc = dual_norms_async(&m, dt, r_dev, d_tmp, d_tmp + 2 * m.ne, (hipStream_t)stream);
  if (rc == STDG_OK) {
    hipError_t e = hipMemcpyAsync(norms_out, d_tmp + 2 * m.ne, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) rc = hip_fail(e, "stdg_residual_dual_norm");
  }
  dev_free(m.ctx, d_tmp, nb);
  return rc;
}

int stdg_energy(const stdg_mesh* mesh, const double* state_dev, double* energy_out, void* stream) {
  if (!mesh || !state_dev || !energy_out) return fail(STDG_E_ARG, "stdg_energy: NULL argument");
  Mesh& m = const_cast<stdg_mesh*>(mesh)->m;
  int rc = ensure_state_off(&m);
  if (rc != STDG_OK) return rc;
  double* d_tmp = nullptr;
  const size_t nb = sizeof(double) * (m.ne + 1);
  if ((rc = dev_alloc(m.ctx, (void**)&d_tmp, nb)) != STDG_OK) return rc;
  rc = energy_async(&m, state_dev, d_tmp, d_tmp + m.ne, (hipStream_t)stream);
  if (rc == STDG_OK) {
    hipError_t e = hipMemcpyAsync(energy_out, d_tmp + m.ne, sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) rc = hip_fail(e, "stdg_energy");
  }
  dev_free(m.ctx, d_tmp, nb);
  return rc;
}

}  // extern "C"
