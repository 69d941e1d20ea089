// Mesh builder: faces, neighbours and their orientations, affine detection,
// metric coefficients, (p, q, affine) groups in locality order, offsets, and
// the device copies (Section 2.2-2.4 of the paper: hexahedral triangulation,
// covariant element maps, interior / boundary faces).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <tuple>

#include "internal.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

namespace stdg {

namespace {

// the 4 local vertices of face (alpha, side), ordered by the tangential
// reference coordinates (u = smaller remaining axis, fastest)
std::array<int, 4> face_local_vertices(int face) {
  int alpha = face / 2, side = face % 2;
  int t0 = alpha == 0 ? 1 : 0;
  int t1 = alpha == 2 ? 1 : 2;
  std::array<int, 4> out{};
  int n = 0;
  for (int bv = 0; bv < 2; ++bv)
    for (int bu = 0; bu < 2; ++bu) {
      int b[3] = {0, 0, 0};
      b[alpha] = side;
      b[t0] = bu;
      b[t1] = bv;
      out[n++] = b[0] + 2 * b[1] + 4 * b[2];
    }
  return out;
}

// Orientation byte (see ElemInfo) of face `face` of element `h` against face
// `face_o` of its neighbour `ho`, from the vertex ids: corner (bu, bv) of our
// face is matched with corner (bu', bv') of theirs; the match must be a
// symmetry of the square.  Returns false if it is not.
bool face_orientation(const int64_t* h, int face, const int64_t* ho, int face_o, uint8_t* out) {
  auto lv = face_local_vertices(face), lo = face_local_vertices(face_o);
  int cu[4], cv[4];
  for (int k = 0; k < 4; ++k) {
    int j = -1;
    for (int l = 0; l < 4; ++l)
      if (ho[lo[l]] == h[lv[k]]) j = l;
    if (j < 0) return false;
    cu[k] = j & 1;
    cv[k] = j >> 1;
  }
  // corner k = bu + 2 bv of our face sits at (cu[k], cv[k]) on theirs
  const bool swap = cu[1] == cu[0];  // moving along our u changes their v'
  int flip_u, flip_v;
  if (!swap) {
    flip_u = cu[0];
    flip_v = cv[0];
  } else {
    flip_u = cv[0];
    flip_v = cu[0];
  }
  // check all four corners against the map
  for (int k = 0; k < 4; ++k) {
    const int bu = k & 1, bv = k >> 1;
    const int ou = swap ? (bv ^ flip_v) : (bu ^ flip_u);
    const int ov = swap ? (bu ^ flip_u) : (bv ^ flip_v);
    if (cu[k] != ou || cv[k] != ov) return false;
  }
  *out = (uint8_t)(face_o | (swap ? kOrientSwap : 0) | (flip_u ? kOrientFlipU : 0) | (flip_v ? kOrientFlipV : 0));
  return true;
}

struct FaceRec {
  std::array<int64_t, 4> key;
  int64_t elem;
  int32_t face;
  bool operator<(const FaceRec& o) const {
    if (key != o.key) return key < o.key;
    if (elem != o.elem) return elem < o.elem;
    return face < o.face;
  }
};

void inv3(const double A[3][3], double B[3][3], double* det_out) {
  double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
               A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
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
  *det_out = det;
}

// G = |J| DF^{-1} DF^{-T} (symmetric) packed xx yy zz xy xz yz
void metric_of(const double DF[3][3], double G[6], double* det) {
  double Di[3][3];
  inv3(DF, Di, det);
  double M[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += Di[i][k] * Di[j][k];
      M[i][j] = *det * s;
    }
  G[0] = M[0][0]; G[1] = M[1][1]; G[2] = M[2][2];
  G[3] = M[0][1]; G[4] = M[0][2]; G[5] = M[1][2];
}

// smallest eigenvalue of a symmetric 3x3 (packed xx yy zz xy xz yz), by the
// trigonometric solution of the characteristic cubic
double sym_lambda_min(const double G[6]) {
  const double p1 = G[3] * G[3] + G[4] * G[4] + G[5] * G[5];
  const double q = (G[0] + G[1] + G[2]) / 3.0;
  if (p1 == 0.0) return std::min(G[0], std::min(G[1], G[2]));
  const double p2 = (G[0] - q) * (G[0] - q) + (G[1] - q) * (G[1] - q) + (G[2] - q) * (G[2] - q) + 2.0 * p1;
  const double p = std::sqrt(p2 / 6.0);
  const double B[6] = {(G[0] - q) / p, (G[1] - q) / p, (G[2] - q) / p, G[3] / p, G[4] / p, G[5] / p};
  const double detB = B[0] * (B[1] * B[2] - B[5] * B[5]) - B[3] * (B[3] * B[2] - B[5] * B[4]) +
                      B[4] * (B[3] * B[5] - B[1] * B[4]);
  const double r = std::max(-1.0, std::min(1.0, detB / 2.0));
  const double phi = std::acos(r) / 3.0;
  return q + 2.0 * p * std::cos(phi + 2.0 * M_PI / 3.0);
}

void sym_inverse(const double G[6], double out[6]) {
  double A[3][3] = {{G[0], G[3], G[4]}, {G[3], G[1], G[5]}, {G[4], G[5], G[2]}};
  double B[3][3], det;
  inv3(A, B, &det);
  out[0] = B[0][0]; out[1] = B[1][1]; out[2] = B[2][2];
  out[3] = B[0][1]; out[4] = B[0][2]; out[5] = B[1][2];
}

uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

}  // namespace

// Work-list orders of the kernel groups.  Morton (order 0): the elements of
// a group sorted along the Morton curve of their centroids.  Columns (order
// T >= 2): columns of T x T elements (on the lattice of the median element
// size) swept along z, the columns in snake order and each swept opposite to
// the previous one, so a neighbour lies at most T^2 elements back or ahead in
// the list; while one XCD's L2 (4 MiB) holds several such layers of element
// blocks nearly every neighbour block read is an L2 hit (Morton order leaves
// about an eighth of the neighbour pairs far apart).  Measured on the 32^3
// p = 4 q = 3 cavity: columns of 8, -5% apply time; no gain for blocks of
// p = 6 q = 4, a loss for several groups (which run concurrently and
// interleave in space).  default_work_order encodes that; stdg_mesh_autotune
// measures instead.
int default_work_order(const Mesh& m) {
  if (m.groups.size() != 1) return 0;
  const int64_t a = m.p[0] + 1;
  const double block = 24.0 * m.q[0] * (double)(a * a * a);  // FP32 bytes of an element's unknowns
  return 4.0 * 1048576.0 / block >= 6.0 * 64.0 ? 8 : 0;
}

int set_work_order(Mesh* m, int order) {
  if (order != 0 && (order < 2 || order > 64)) return fail(STDG_E_ARG, "work order must be 0 (Morton) or 2..64");
  ++m->epoch;
  const int64_t ne = m->ne;
  std::vector<std::array<double, 3>> cen(ne);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t e = 0; e < ne; ++e)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int v = 0; v < 8; ++v) s += m->verts[24 * e + 3 * v + c];
      cen[e][c] = s / 8.0;
      lo[c] = std::min(lo[c], cen[e][c]);
      hi[c] = std::max(hi[c], cen[e][c]);
    }
  std::function<uint64_t(int64_t)> key;
  double h[3] = {1.0, 1.0, 1.0};
  int64_t ntx = 1;
  const int64_t T = order;
  auto cell = [&](int64_t e, int c) {
    return (int64_t)std::max(0.0, std::min(1048575.0, std::floor((cen[e][c] - lo[c]) / h[c] + 0.5)));
  };
  if (order == 0) {
    key = [&](int64_t e) {
      uint64_t code = 0;
      for (int c = 0; c < 3; ++c) {
        const double span = hi[c] - lo[c];
        const double t = span > 0 ? (cen[e][c] - lo[c]) / span : 0.0;
        const uint64_t iv = (uint64_t)std::min(1048575.0, std::max(0.0, std::floor(t * 1048575.0)));
        code |= spread3(iv) << c;
      }
      return code;
    };
  } else {
    for (int c = 0; c < 3; ++c) {
      std::vector<double> ext(ne);
      for (int64_t e = 0; e < ne; ++e) {
        double a = 1e300, b = -1e300;
        for (int v = 0; v < 8; ++v) {
          a = std::min(a, m->verts[24 * e + 3 * v + c]);
          b = std::max(b, m->verts[24 * e + 3 * v + c]);
        }
        ext[e] = b - a;
      }
      std::nth_element(ext.begin(), ext.begin() + ne / 2, ext.end());
      h[c] = ext[ne / 2] > 0 ? ext[ne / 2] : 1.0;
    }
    for (int64_t e = 0; e < ne; ++e) ntx = std::max(ntx, cell(e, 0) / T + 1);
    key = [&](int64_t e) {
      const int64_t ix = cell(e, 0), iy = cell(e, 1), iz = cell(e, 2);
      const int64_t tx = ix / T, ty = iy / T;
      const int64_t tile = ty * ntx + ((ty & 1) ? ntx - 1 - tx : tx);
      const int64_t zz = (tile & 1) ? 1048575 - iz : iz;
      return ((uint64_t)tile << 40) | ((uint64_t)zz << 20) | (uint64_t)((iy % T) * T + (ix % T));
    };
  }
  for (Group& g : m->groups) {
    std::vector<std::pair<uint64_t, int32_t>> lst(g.ids.size());
    for (size_t i = 0; i < g.ids.size(); ++i) lst[i] = {key(g.ids[i]), g.ids[i]};
    std::sort(lst.begin(), lst.end());
    for (size_t i = 0; i < lst.size(); ++i) g.ids[i] = lst[i].second;
    if (g.d_list)
      STDG_HIP(hipMemcpy(g.d_list, g.ids.data(), sizeof(int32_t) * g.count, hipMemcpyHostToDevice));
  }
  m->work_order = order;
  return STDG_OK;
}

int build_mesh_host(const stdg_mesh_desc* d, Mesh* m) {
  const int64_t ne = d->n_elements, nv = d->n_vertices;
  m->ne = ne;
  m->nv = nv;
  m->p.assign(d->p, d->p + ne);
  m->q.assign(d->q, d->q + ne);
  if (d->nsub) m->nsub.assign(d->nsub, d->nsub + ne); else m->nsub.assign(ne, 1);
  for (int64_t e = 0; e < ne; ++e) {
    if (m->p[e] < 1 || m->p[e] > kMaxA - 1)
      return fail(STDG_E_ARG, "element " + std::to_string(e) + ": p must be in 1..8");
    if (m->q[e] < 1 || m->q[e] > kMaxQ)
      return fail(STDG_E_ARG, "element " + std::to_string(e) + ": q must be in 1..6");
    const int32_t ns = m->nsub[e];
    if (ns < 1 || ns > kMaxSub || (ns & (ns - 1)))
      return fail(STDG_E_ARG, "element " + std::to_string(e) + ": sub-intervals must be 1, 2, 4 or 8");
    if (ns > 1 && ns * m->q[e] > kMaxLocalLevels)
      return fail(STDG_E_ARG, "element " + std::to_string(e) + ": sub-intervals times q must be <= 24");
    if (!(d->eps[e] > 0.0) || !(d->mu[e] > 0.0) || !std::isfinite(d->eps[e]) || !std::isfinite(d->mu[e]))
      return fail(STDG_E_ARG, "element " + std::to_string(e) + ": eps and mu must be finite and > 0");
    for (int v = 0; v < 8; ++v) {
      int64_t id = d->hexes[8 * e + v];
      if (id < 0 || id >= nv) return fail(STDG_E_ARG, "element " + std::to_string(e) + ": vertex id out of range");
    }
  }
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(d->vertices[i])) return fail(STDG_E_ARG, "non-finite vertex coordinate");

  // offsets
  m->trial_off.assign(ne + 1, 0);
  m->unk_off.assign(ne + 1, 0);
  m->state_off.assign(ne + 1, 0);
  for (int64_t e = 0; e < ne; ++e) {
    int64_t a3 = (int64_t)(m->p[e] + 1) * (m->p[e] + 1) * (m->p[e] + 1);
    const int64_t nl = (int64_t)m->q[e] * m->nsub[e];  // test levels; trial levels nl + 1
    m->trial_off[e + 1] = m->trial_off[e] + 6 * (nl + 1) * a3;
    m->unk_off[e + 1] = m->unk_off[e] + 6 * nl * a3;
    m->state_off[e + 1] = m->state_off[e] + 6 * a3;
  }

  // faces
  std::vector<FaceRec> faces;
  faces.reserve(6 * ne);
  for (int64_t e = 0; e < ne; ++e)
    for (int f = 0; f < 6; ++f) {
      auto lv = face_local_vertices(f);
      FaceRec r;
      for (int k = 0; k < 4; ++k) r.key[k] = d->hexes[8 * e + lv[k]];
      std::sort(r.key.begin(), r.key.end());
      r.elem = e;
      r.face = f;
      faces.push_back(r);
    }
  std::sort(faces.begin(), faces.end());
  m->info.assign(ne, ElemInfo{});
  for (int64_t e = 0; e < ne; ++e) {
    ElemInfo& I = m->info[e];
    I.a = m->p[e] + 1;
    I.q = m->q[e];
    I.nsub = (uint8_t)m->nsub[e];
    I.flags = 0;
    I.trial_off = m->trial_off[e];
    I.unk_off = m->unk_off[e];
    for (int f = 0; f < 6; ++f) I.nb[f] = -1;
  }
  m->n_int_faces = m->n_bnd_faces = 0;
  for (size_t i = 0; i < faces.size();) {
    size_t j = i + 1;
    while (j < faces.size() && faces[j].key == faces[i].key) ++j;
    if (j - i == 1) {
      m->info[faces[i].elem].flags |= (kBoundaryBase << faces[i].face);
      ++m->n_bnd_faces;
    } else if (j - i == 2) {
      const FaceRec &A = faces[i], &B = faces[i + 1];
      if (A.elem == B.elem) return fail(STDG_E_ARG, "element touches itself across a face");
      if (A.elem > INT32_MAX || B.elem > INT32_MAX) return fail(STDG_E_ARG, "too many elements");
      uint8_t oa, ob;
      if (!face_orientation(d->hexes + 8 * A.elem, A.face, d->hexes + 8 * B.elem, B.face, &oa) ||
          !face_orientation(d->hexes + 8 * B.elem, B.face, d->hexes + 8 * A.elem, A.face, &ob))
        return fail(STDG_E_ARG, "face between elements " + std::to_string(A.elem) + " and " +
                                    std::to_string(B.elem) + " does not match as a quadrilateral");
      m->info[A.elem].nb[A.face] = (int32_t)B.elem;
      m->info[B.elem].nb[B.face] = (int32_t)A.elem;
      m->info[A.elem].orient[A.face] = oa;
      m->info[B.elem].orient[B.face] = ob;
      if (oa != (uint8_t)(A.face ^ 1)) m->info[A.elem].flags |= kPermuted;
      if (ob != (uint8_t)(B.face ^ 1)) m->info[B.elem].flags |= kPermuted;
      ++m->n_int_faces;
    } else {
      return fail(STDG_E_ARG, "non-manifold face shared by more than two elements");
    }
    i = j;
  }

  // 2:1 hanging faces: a coarse face and the four fine faces covering it
  // are left unmatched above.  Such a coarse face has mesh vertices at its
  // edge midpoints and centre (the bilinear face map at (i/2, j/2)), and its
  // quarters are unmatched faces of four other elements with those vertex
  // ids (positions compared with a spatial hash, tolerance 1e-9 of the mesh
  // size).  Both sides are recorded (HangRec) and the faces become interior.
  {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < nv; ++v)
      for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(lo[c], d->vertices[3 * v + c]);
        hi[c] = std::max(hi[c], d->vertices[3 * v + c]);
      }
    const double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                  (hi[2] - lo[2]) * (hi[2] - lo[2]));
    const double tol = 1e-9 * (diag > 0 ? diag : 1.0);
    auto cell = [&](const double* x, int c) { return (int64_t)std::floor((x[c] - lo[c]) / (4 * tol)); };
    std::map<std::array<int64_t, 3>, std::vector<int64_t>> vgrid;
    for (int64_t v = 0; v < nv; ++v) {
      const double* x = d->vertices + 3 * v;
      vgrid[{cell(x, 0), cell(x, 1), cell(x, 2)}].push_back(v);
    }
    auto vertex_at = [&](const double x[3]) -> int64_t {
      const int64_t c0 = cell(x, 0), c1 = cell(x, 1), c2 = cell(x, 2);
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            auto it = vgrid.find({c0 + dx, c1 + dy, c2 + dz});
            if (it == vgrid.end()) continue;
            for (int64_t v : it->second) {
              const double* y = d->vertices + 3 * v;
              if (std::fabs(y[0] - x[0]) <= tol && std::fabs(y[1] - x[1]) <= tol && std::fabs(y[2] - x[2]) <= tol)
                return v;
            }
          }
      return -1;
    };
    // unmatched faces by their sorted vertex ids
    std::map<std::array<int64_t, 4>, std::pair<int64_t, int>> open;
    for (int64_t e = 0; e < ne; ++e)
      for (int f = 0; f < 6; ++f) {
        if (m->info[e].nb[f] >= 0) continue;
        auto lv = face_local_vertices(f);
        std::array<int64_t, 4> key;
        for (int k = 0; k < 4; ++k) key[k] = d->hexes[8 * e + lv[k]];
        std::sort(key.begin(), key.end());
        open[key] = {e, f};
      }
    auto record = [&](int64_t e) -> HangRec& {
      ElemInfo& I = m->info[e];
      if (!(I.flags & kHanging)) {
        I.flags |= kHanging;
        I.pad = (int32_t)m->hang.size();
        HangRec r;
        std::memset(&r, 0, sizeof(r));
        r.elem = (int32_t)e;
        m->hang.push_back(r);
      }
      return m->hang[I.pad];
    };
    for (int64_t e = 0; e < ne; ++e)
      for (int f = 0; f < 6; ++f) {
        if (m->info[e].nb[f] >= 0) continue;
        if ((m->info[e].flags & kHanging) && m->hang[m->info[e].pad].f[f].kind != 0) continue;
        auto lv = face_local_vertices(f);  // corners (0,0), (1,0), (0,1), (1,1)
        int64_t grid[3][3];
        bool ok = true;
        for (int j = 0; j < 3 && ok; ++j)
          for (int i = 0; i < 3 && ok; ++i) {
            const double s_ = 0.5 * i, t_ = 0.5 * j;
            const double wt[4] = {(1 - s_) * (1 - t_), s_ * (1 - t_), (1 - s_) * t_, s_ * t_};
            double x[3] = {0, 0, 0};
            for (int k = 0; k < 4; ++k)
              for (int c = 0; c < 3; ++c) x[c] += wt[k] * d->vertices[3 * d->hexes[8 * e + lv[k]] + c];
            grid[i][j] = vertex_at(x);
            ok = grid[i][j] >= 0;
          }
        if (!ok) continue;
        std::pair<int64_t, int> fine[4];
        for (int qd = 0; qd < 4 && ok; ++qd) {
          const int hu = qd & 1, hv = qd >> 1;
          std::array<int64_t, 4> key = {grid[hu][hv], grid[hu + 1][hv], grid[hu][hv + 1], grid[hu + 1][hv + 1]};
          std::sort(key.begin(), key.end());
          auto it = open.find(key);
          ok = it != open.end() && it->second.first != e;
          if (ok) fine[qd] = it->second;
        }
        if (!ok) continue;
        if (m->info[e].q < 1) return fail(STDG_E_ARG, "hanging face: invalid element");
        HangFace hc;
        std::memset(&hc, 0, sizeof(hc));
        hc.kind = 1;
        for (int qd = 0; qd < 4; ++qd) {
          const int64_t k = fine[qd].first;
          const int fk = fine[qd].second;
          if (k > INT32_MAX || e > INT32_MAX) return fail(STDG_E_ARG, "too many elements");
          // the fine face's corners in the coarse face's coordinates (halves)
          auto fv = face_local_vertices(fk);
          int cu[4], cv[4];
          for (int t = 0; t < 4; ++t) {
            const int64_t g = d->hexes[8 * k + fv[t]];
            cu[t] = cv[t] = -1;
            for (int j = 0; j < 3; ++j)
              for (int i = 0; i < 3; ++i)
                if (grid[i][j] == g) {
                  cu[t] = i;
                  cv[t] = j;
                }
            if (cu[t] < 0) return fail(STDG_E_ARG, "hanging face: a fine face does not match its quarter");
          }
          // fine (u, v) -> coarse (2u', 2v') = A (u, v) + b (entries of A: 0, +-1 in half units)
          const int A00 = cu[1] - cu[0], A10 = cv[1] - cv[0], A01 = cu[2] - cu[0], A11 = cv[2] - cv[0];
          if (cu[3] != cu[0] + A00 + A01 || cv[3] != cv[0] + A10 + A11 || std::abs(A00) + std::abs(A01) != 1 ||
              std::abs(A10) + std::abs(A11) != 1 || std::abs(A00) + std::abs(A10) != 1)
            return fail(STDG_E_ARG, "hanging face: a fine face does not match its quarter as a quadrilateral");
          const bool swap = A00 == 0;
          // fine side: the coarse coordinate matched with fine u is u' (or v' when swapped)
          const bool fu_flip = swap ? A10 < 0 : A00 < 0;
          const bool fv_flip = swap ? A01 < 0 : A11 < 0;
          const int wu0 = swap ? cv[0] : cu[0], wv0 = swap ? cu[0] : cv[0];  // in half units at fine (0, 0)
          const int hu_f = wu0 - (fu_flip ? 1 : 0), hv_f = wv0 - (fv_flip ? 1 : 0);
          if (hu_f < 0 || hu_f > 1 || hv_f < 0 || hv_f > 1) return fail(STDG_E_ARG, "hanging face: bad quarter");
          HangRec& rf = record(k);
          HangFace& hf = rf.f[fk];
          hf.kind = 2;
          hf.nb[0] = (int32_t)e;
          hf.code[0] = (uint8_t)(f | (swap ? 8 : 0) | (fu_flip ? 16 : 0) | (fv_flip ? 32 : 0) | (hu_f << 6) | (hv_f << 7));
          // coarse side: the inverse map, 2 times the transposed signed permutation
          const int B00 = A00, B01 = A10, B10 = A01, B11 = A11;  // P^T (P is a signed permutation)
          const bool cswap = B00 == 0;
          const bool cu_flip = cswap ? B10 < 0 : B00 < 0;
          const bool cv_flip = cswap ? B01 < 0 : B11 < 0;
          const int qu = std::min(std::min(cu[0], cu[1]), std::min(cu[2], cu[3]));
          const int qv = std::min(std::min(cv[0], cv[1]), std::min(cv[2], cv[3]));
          const int slot = qu + 2 * qv;
          hc.nb[slot] = (int32_t)k;
          hc.code[slot] = (uint8_t)(fk | (cswap ? 8 : 0) | (cu_flip ? 16 : 0) | (cv_flip ? 32 : 0));
          m->info[k].nb[fk] = (int32_t)e;
          m->info[k].orient[fk] = (uint8_t)(fk ^ 1);
          m->info[k].flags &= ~(kBoundaryBase << fk);
          m->info[k].flags |= (kHangFaceBase << fk);
        }
        HangRec& rc = record(e);
        rc.f[f] = hc;
        m->info[e].nb[f] = hc.nb[0];
        m->info[e].orient[f] = (uint8_t)(f ^ 1);
        m->info[e].flags &= ~(kBoundaryBase << f);
        m->info[e].flags |= (kHangFaceBase << f);
        m->n_hanging_faces += 1;
        m->n_bnd_faces -= 5;
        m->n_int_faces += 4;
      }
  }

  // a face split among smaller elements that did not match as a 2:1 hanging
  // face above (its quarters are not whole faces with the corner, edge-midpoint
  // and centre vertices of the face's bilinear map) would be taken for a wall:
  // refuse it.  Such a face has the centroids of the smaller faces at its
  // quarter points: look every remaining boundary face's quarter points up
  // among the boundary-face centroids (spatial hash, tolerance 1e-9 of the
  // mesh size).
  {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < nv; ++v)
      for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(lo[c], d->vertices[3 * v + c]);
        hi[c] = std::max(hi[c], d->vertices[3 * v + c]);
      }
    const double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                  (hi[2] - lo[2]) * (hi[2] - lo[2]));
    const double tol = 1e-9 * (diag > 0 ? diag : 1.0);
    auto point = [&](int64_t e, int f, double u, double w, double out[3]) {
      auto lv = face_local_vertices(f);  // corners (0,0), (1,0), (0,1), (1,1)
      const double wt[4] = {(1 - u) * (1 - w), u * (1 - w), (1 - u) * w, u * w};
      for (int c = 0; c < 3; ++c) {
        out[c] = 0.0;
        for (int k = 0; k < 4; ++k) out[c] += wt[k] * d->vertices[3 * d->hexes[8 * e + lv[k]] + c];
      }
    };
    auto cell = [&](const double x[3], int c) { return (int64_t)std::floor((x[c] - lo[c]) / (4 * tol)); };
    std::map<std::array<int64_t, 3>, std::vector<std::array<double, 3>>> grid;
    for (int64_t e = 0; e < ne; ++e)
      for (int f = 0; f < 6; ++f) {
        if (m->info[e].nb[f] >= 0) continue;
        double x[3];
        point(e, f, 0.5, 0.5, x);
        grid[{cell(x, 0), cell(x, 1), cell(x, 2)}].push_back({x[0], x[1], x[2]});
      }
    for (int64_t e = 0; e < ne; ++e)
      for (int f = 0; f < 6; ++f) {
        if (m->info[e].nb[f] >= 0) continue;
        for (int k = 0; k < 4; ++k) {
          double x[3];
          point(e, f, (k & 1) ? 0.75 : 0.25, (k & 2) ? 0.75 : 0.25, x);
          const int64_t c0 = cell(x, 0), c1 = cell(x, 1), c2 = cell(x, 2);
          for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx) {
                auto it = grid.find({c0 + dx, c1 + dy, c2 + dz});
                if (it == grid.end()) continue;
                for (const auto& y : it->second)
                  if (std::fabs(y[0] - x[0]) <= tol && std::fabs(y[1] - x[1]) <= tol && std::fabs(y[2] - x[2]) <= tol)
                    return fail(STDG_E_UNSUPPORTED, "nonconforming mesh: face " + std::to_string(f) + " of element " +
                                                        std::to_string(e) +
                                                        " is split among smaller elements that are not its four quarters");
              }
        }
      }
  }

  // geometry
  m->metric.assign(ne, ElemMetric{});
  m->verts.assign(ne * 24, 0.0);
  m->n_affine = m->n_nonaffine = m->n_diag = 0;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  std::vector<std::array<double, 3>> cen(ne);
  for (int64_t e = 0; e < ne; ++e) {
    double X[8][3];
    for (int v = 0; v < 8; ++v)
      for (int c = 0; c < 3; ++c) {
        X[v][c] = d->vertices[3 * d->hexes[8 * e + v] + c];
        m->verts[24 * e + 3 * v + c] = X[v][c];
      }
    double scale = 0.0;
    for (int v = 0; v < 8; ++v)
      for (int c = 0; c < 3; ++c) scale = std::max(scale, std::fabs(X[v][c] - X[0][c]));
    bool affine = true;
    for (int v = 0; v < 8; ++v) {
      int b0 = v & 1, b1 = (v >> 1) & 1, b2 = (v >> 2) & 1;
      for (int c = 0; c < 3; ++c) {
        double pred = X[0][c] + b0 * (X[1][c] - X[0][c]) + b1 * (X[2][c] - X[0][c]) + b2 * (X[4][c] - X[0][c]);
        if (std::fabs(pred - X[v][c]) > 1e-12 * scale) affine = false;
      }
    }
    // DF at the element centre (exact for affine elements)
    double DF[3][3] = {{0}};
    for (int v = 0; v < 8; ++v) {
      int b[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
      for (int mdir = 0; mdir < 3; ++mdir) {
        double dN = (b[mdir] ? 1.0 : -1.0) * 0.25;
        for (int c = 0; c < 3; ++c) DF[c][mdir] += dN * X[v][c];
      }
    }
    double G[6], det;
    metric_of(DF, G, &det);
    if (!(det > 0.0)) return fail(STDG_E_ARG, "element " + std::to_string(e) + " is inverted or degenerate");
    // the trilinear map's Jacobian at each corner is the matrix of the three
    // edges leaving it (oriented along the reference axes): all must be > 0
    for (int v = 0; v < 8; ++v) {
      double J[3][3];
      for (int ax = 0; ax < 3; ++ax) {
        const int w = v ^ (1 << ax);
        const double sgn = ((v >> ax) & 1) ? -1.0 : 1.0;
        for (int c = 0; c < 3; ++c) J[c][ax] = sgn * (X[w][c] - X[v][c]);
      }
      const double dj = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      if (!(dj > 0.0))
        return fail(STDG_E_ARG, "element " + std::to_string(e) + " is inverted or folded at corner " + std::to_string(v));
    }
    ElemMetric& M = m->metric[e];
    M.eps = d->eps[e];
    M.mu = d->mu[e];
    for (int k = 0; k < 6; ++k) {
      M.m[k] = d->eps[e] * G[k];
      M.m[6 + k] = d->mu[e] * G[k];
    }
    sym_inverse(M.m, M.m + 12);
    sym_inverse(M.m + 6, M.m + 18);
    // with n sub-intervals a test function lives on dt / n: the dual-norm bound scales by n
    m->inv_gmin = std::max(m->inv_gmin, m->nsub[e] / sym_lambda_min(G));
    m->eps_min = e == 0 ? d->eps[e] : std::min(m->eps_min, d->eps[e]);
    m->mu_min = e == 0 ? d->mu[e] : std::min(m->mu_min, d->mu[e]);
    bool diag = affine && std::fabs(G[3]) <= 1e-13 * (G[0] + G[1] + G[2]) &&
                std::fabs(G[4]) <= 1e-13 * (G[0] + G[1] + G[2]) && std::fabs(G[5]) <= 1e-13 * (G[0] + G[1] + G[2]);
    if (diag) {
      M.m[3] = M.m[4] = M.m[5] = M.m[9] = M.m[10] = M.m[11] = 0.0;
      M.m[15] = M.m[16] = M.m[17] = M.m[21] = M.m[22] = M.m[23] = 0.0;
    }
    ElemInfo& I = m->info[e];
    if (affine) { I.flags |= kAffine; ++m->n_affine; } else { ++m->n_nonaffine; }
    if (diag) { I.flags |= kDiagMass; ++m->n_diag; }
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int v = 0; v < 8; ++v) s += X[v][c];
      cen[e][c] = s / 8.0;
      lo[c] = std::min(lo[c], cen[e][c]);
      hi[c] = std::max(hi[c], cen[e][c]);
    }
  }

  // neighbours must lie across the face: the neighbour's centroid on the
  // outer side of the face (refuses coincident or folded elements)
  for (int64_t e = 0; e < ne; ++e)
    for (int f = 0; f < 6; ++f) {
      const int32_t k = m->info[e].nb[f];
      if (k < 0) continue;
      auto lv = face_local_vertices(f);
      double fc[3] = {0, 0, 0};
      for (int t = 0; t < 4; ++t)
        for (int c = 0; c < 3; ++c) fc[c] += 0.25 * m->verts[24 * e + 3 * lv[t] + c];
      double out = 0.0, ref = 0.0;
      for (int c = 0; c < 3; ++c) {
        out += (cen[k][c] - fc[c]) * (fc[c] - cen[e][c]);
        ref += (fc[c] - cen[e][c]) * (fc[c] - cen[e][c]);
      }
      if (!(out > 1e-12 * ref))
        return fail(STDG_E_ARG, "elements " + std::to_string(e) + " and " + std::to_string(k) +
                                    " share a face but do not lie on its two sides");
    }

  // local time steps: the rows of elements with several sub-intervals, and of
  // their face neighbours (whose coupling then runs through the projection
  // onto a piecewise common test space), leave the kernel groups for the
  // local-time kernel
  m->lt.clear();
  m->lt_work.clear();
  m->lt_bank.clear();
  if (*std::max_element(m->nsub.begin(), m->nsub.end()) > 1) {
    if (!m->hang.empty()) return fail(STDG_E_UNSUPPORTED, "local time steps on meshes with 2:1 hanging faces");
    std::map<std::pair<int, int>, std::pair<int32_t, int32_t>> own;
    std::map<std::tuple<int, int, int, int>, int32_t> cpl, prj;
    for (int64_t e = 0; e < ne; ++e) {
      ElemInfo& I = m->info[e];
      bool local = m->nsub[e] > 1;
      for (int f = 0; f < 6; ++f)
        if (I.nb[f] >= 0 && m->nsub[I.nb[f]] > 1) local = true;
      if (!local) continue;
      if (!(I.flags & kAffine))
        return fail(STDG_E_UNSUPPORTED, "element " + std::to_string(e) +
                                            ": local time steps need affine elements (and their face neighbours)");
      LTRec R;
      R.elem = (int32_t)e;
      auto ok = own.find({m->q[e], m->nsub[e]});
      if (ok == own.end()) {
        int32_t d_off, n_off;
        local_time_tables(m->q[e], m->nsub[e], &m->lt_bank, &d_off, &n_off);
        ok = own.emplace(std::make_pair(m->q[e], m->nsub[e]), std::make_pair(d_off, n_off)).first;
      }
      R.d_off = ok->second.first;
      R.n_off = ok->second.second;
      for (int f = 0; f < 6; ++f) {
        R.c_off[f] = -1;
        R.s_off[f] = -1;
        const int32_t k = I.nb[f];
        if (k < 0) continue;
        {
          const int r = std::min(m->q[e], m->q[k]), npj = std::min(m->nsub[e], m->nsub[k]);
          auto pk = std::make_tuple(m->q[e], m->nsub[e], r, npj);
          auto pt = prj.find(pk);
          if (pt == prj.end())
            pt = prj.emplace(pk, local_projected_table(m->q[e], m->nsub[e], r, npj, &m->lt_bank)).first;
          R.s_off[f] = pt->second;
        }
        auto key = std::make_tuple(m->q[e], m->nsub[e], m->q[k], m->nsub[k]);
        auto it = cpl.find(key);
        if (it == cpl.end())
          it = cpl.emplace(key, local_coupling_table(m->q[e], m->nsub[e], m->q[k], m->nsub[k], &m->lt_bank)).first;
        R.c_off[f] = it->second;
      }
      I.flags |= kLocalTime;
      I.pad = (int32_t)m->lt.size();
      for (int j = 0; j < m->nsub[e]; ++j) m->lt_work.push_back((int32_t)m->lt.size() * kMaxSub + j);
      m->lt.push_back(R);
    }
    // the local-time kernel is instantiated per a: group its work by a
    std::stable_sort(m->lt_work.begin(), m->lt_work.end(), [&](int32_t x, int32_t y) {
      return m->info[m->lt[x / kMaxSub].elem].a < m->info[m->lt[y / kMaxSub].elem].a;
    });
  }
  m->lt_a_off.assign(kMaxA + 2, 0);
  m->lt_a_qmax.assign(kMaxA + 2, 1);
  for (int32_t w : m->lt_work) {
    const ElemInfo& I = m->info[m->lt[w / kMaxSub].elem];
    ++m->lt_a_off[I.a + 1];
    m->lt_a_qmax[I.a] = std::max(m->lt_a_qmax[I.a], I.q);
  }
  for (int a = 1; a <= kMaxA + 1; ++a) m->lt_a_off[a] += m->lt_a_off[a - 1];

  // kernel groups by (a, q, affine); their work-list order is set below
  std::map<std::tuple<int, int, int>, std::vector<std::pair<uint64_t, int32_t>>> gm;
  for (int64_t e = 0; e < ne; ++e) {
    if (m->info[e].flags & kLocalTime) continue;
    auto key = std::make_tuple(m->p[e] + 1, m->q[e], (m->info[e].flags & kAffine) ? 1 : 0);
    gm[key].push_back({0, (int32_t)e});
  }
  m->p_max = *std::max_element(m->p.begin(), m->p.end());
  m->q_max = *std::max_element(m->q.begin(), m->q.end());
  m->groups.clear();
  for (auto& kv : gm) {
    auto& lst = kv.second;
    std::sort(lst.begin(), lst.end());
    Group g;
    g.a = std::get<0>(kv.first);
    g.q = std::get<1>(kv.first);
    g.affine = std::get<2>(kv.first);
    g.count = (int64_t)lst.size();
    g.d_list = nullptr;
    g.ids.resize(lst.size());
    for (size_t i = 0; i < lst.size(); ++i) g.ids[i] = lst[i].second;
    m->groups.push_back(std::move(g));
  }
  return set_work_order(m, default_work_order(*m));
}

size_t mesh_device_bytes(const Mesh& m) {
  auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t b = r256(sizeof(ElemInfo) * m.ne) + r256(sizeof(ElemMetric) * m.ne) + r256(sizeof(double) * 24 * m.ne) +
             r256(sizeof(QTables<double>) * (kMaxA + 1)) + r256(sizeof(QTables<float>) * (kMaxA + 1)) +
             r256(sizeof(int64_t) * (m.ne + 1));
  if (m.n_nonaffine > 0)
    b += r256(sizeof(FaceRule<double>) * (kMaxFaceQ + 1)) + r256(sizeof(FaceRule<float>) * (kMaxFaceQ + 1));
  if (!m.hang.empty())
    b += r256(sizeof(HangRec) * m.hang.size()) + r256(sizeof(double) * 2 * kMaxA * kMaxA) +
         r256(sizeof(float) * 2 * kMaxA * kMaxA);
  if (!m.lt.empty())
    b += r256(sizeof(LTRec) * m.lt.size()) + r256(sizeof(int32_t) * m.lt_work.size()) +
         r256(sizeof(double) * m.lt_bank.size()) + r256(sizeof(float) * m.lt_bank.size());
  for (const Group& g : m.groups) b += r256(sizeof(int32_t) * g.count);
  return b;
}

int upload_mesh(Ctx* ctx, Mesh* m) {
  const int64_t ne = m->ne;
  m->ctx = ctx;
  // device copies
  size_t bytes_info = sizeof(ElemInfo) * ne, bytes_metric = sizeof(ElemMetric) * ne;
  size_t bytes_verts = sizeof(double) * 24 * ne;
  int rc;
  if ((rc = dev_alloc(ctx, (void**)&m->d_info, bytes_info)) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&m->d_metric, bytes_metric)) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&m->d_verts, bytes_verts)) != STDG_OK) return rc;
  m->device_bytes = bytes_info + bytes_metric + bytes_verts;
  STDG_HIP(hipMemcpy(m->d_info, m->info.data(), bytes_info, hipMemcpyHostToDevice));
  STDG_HIP(hipMemcpy(m->d_metric, m->metric.data(), bytes_metric, hipMemcpyHostToDevice));
  STDG_HIP(hipMemcpy(m->d_verts, m->verts.data(), bytes_verts, hipMemcpyHostToDevice));
  {
    std::vector<QTables<double>> q64(kMaxA + 1);
    std::vector<QTables<float>> q32(kMaxA + 1);
    for (int a = 1; a <= kMaxA; ++a) {
      fill_qtables_f64(a, &q64[a]);
      fill_qtables_f32(a, &q32[a]);
    }
    size_t b64 = sizeof(QTables<double>) * (kMaxA + 1), b32 = sizeof(QTables<float>) * (kMaxA + 1);
    if ((rc = dev_alloc(ctx, &m->d_qt64, b64)) != STDG_OK) return rc;
    if ((rc = dev_alloc(ctx, &m->d_qt32, b32)) != STDG_OK) return rc;
    m->device_bytes += b64 + b32;
    STDG_HIP(hipMemcpy(m->d_qt64, q64.data(), b64, hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d_qt32, q32.data(), b32, hipMemcpyHostToDevice));
  }
  if (m->n_nonaffine > 0) {
    std::vector<FaceRule<double>> f64(kMaxFaceQ + 1);
    std::vector<FaceRule<float>> f32(kMaxFaceQ + 1);
    for (int n = 1; n <= kMaxFaceQ; ++n) {
      fill_face_rule_f64(n, &f64[n]);
      fill_face_rule_f32(n, &f32[n]);
    }
    size_t b64 = sizeof(FaceRule<double>) * (kMaxFaceQ + 1), b32 = sizeof(FaceRule<float>) * (kMaxFaceQ + 1);
    if ((rc = dev_alloc(ctx, &m->d_fr64, b64)) != STDG_OK) return rc;
    if ((rc = dev_alloc(ctx, &m->d_fr32, b32)) != STDG_OK) return rc;
    m->device_bytes += b64 + b32;
    STDG_HIP(hipMemcpy(m->d_fr64, f64.data(), b64, hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d_fr32, f32.data(), b32, hipMemcpyHostToDevice));
  }
  if (!m->hang.empty()) {
    const size_t bh = sizeof(HangRec) * m->hang.size();
    std::vector<double> s64(2 * kMaxA * kMaxA);
    fill_half_tables_f64(s64.data());
    std::vector<float> s32(s64.begin(), s64.end());
    if ((rc = dev_alloc(ctx, (void**)&m->d_hang, bh)) != STDG_OK) return rc;
    if ((rc = dev_alloc(ctx, &m->d_hs64, sizeof(double) * s64.size())) != STDG_OK) return rc;
    if ((rc = dev_alloc(ctx, &m->d_hs32, sizeof(float) * s32.size())) != STDG_OK) return rc;
    m->device_bytes += bh + sizeof(double) * s64.size() + sizeof(float) * s32.size();
    STDG_HIP(hipMemcpy(m->d_hang, m->hang.data(), bh, hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d_hs64, s64.data(), sizeof(double) * s64.size(), hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d_hs32, s32.data(), sizeof(float) * s32.size(), hipMemcpyHostToDevice));
  }
  if (!m->lt.empty()) {
    const size_t bl = sizeof(LTRec) * m->lt.size(), nb = m->lt_bank.size();
    std::vector<float> b32(m->lt_bank.begin(), m->lt_bank.end());
    if ((rc = dev_alloc(ctx, (void**)&m->d_lt, bl)) != STDG_OK) return rc;
    if ((rc = dev_alloc(ctx, (void**)&m->d_lt_work, sizeof(int32_t) * m->lt_work.size())) != STDG_OK) return rc;
    if ((rc = dev_alloc(ctx, &m->d_ltb64, sizeof(double) * nb)) != STDG_OK) return rc;
    if ((rc = dev_alloc(ctx, &m->d_ltb32, sizeof(float) * nb)) != STDG_OK) return rc;
    m->device_bytes += bl + sizeof(int32_t) * m->lt_work.size() + (sizeof(double) + sizeof(float)) * nb;
    STDG_HIP(hipMemcpy(m->d_lt, m->lt.data(), bl, hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d_lt_work, m->lt_work.data(), sizeof(int32_t) * m->lt_work.size(), hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d_ltb64, m->lt_bank.data(), sizeof(double) * nb, hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d_ltb32, b32.data(), sizeof(float) * nb, hipMemcpyHostToDevice));
  }
  for (Group& g : m->groups) {
    if ((rc = dev_alloc(ctx, (void**)&g.d_list, sizeof(int32_t) * g.count)) != STDG_OK) return rc;
    m->device_bytes += sizeof(int32_t) * g.count;
    STDG_HIP(hipMemcpy(g.d_list, g.ids.data(), sizeof(int32_t) * g.count, hipMemcpyHostToDevice));
  }
  return STDG_OK;
}

// Coefficients of D_h (the dissipative remark closing Section 4):
// alpha_E = c / {sqrt(mu / eps)}, alpha_H = c / {sqrt(eps / mu)} per face (the
// mean of both sides, the element's own value on PEC faces, where only the E
// term exists), and per axis the face metric K that turns the physical
// integral of (n x v) . (n x u) into sum K_cd v_c u_d over the reference face
// (constant on affine elements; the trilinear kernels evaluate it at the face
// quadrature points from the vertices and leave these entries unused).
int set_dissipation(Mesh* m, double c) {
  if (!(c >= 0.0) || !std::isfinite(c)) return fail(STDG_E_ARG, "dissipation coefficient must be finite and >= 0");
  if (c > 0.0 && !m->hang.empty())
    return fail(STDG_E_UNSUPPORTED, "dissipative stabilisation on meshes with hanging faces");
  if (c > 0.0 && !m->lt.empty()) {
    // the local-time kernel's LDS with D_h (table rows, contracted fields, face
    // values and jumps) must fit in 64 KB for the largest rows
    for (const LTRec& r : m->lt) {
      const size_t a = (size_t)m->info[r.elem].a, q = (size_t)m->info[r.elem].q;
      const size_t need = (2 * kMaxA + kMaxA * kMaxA + 14 * q * (kMaxLocalLevels + 1) + 6 * a * a * a + 48 * a * a) *
                          sizeof(double);
      if (need > 65536 || (q >= 5 && (int)a > kMaxDissLocalA7))
        return fail(STDG_E_UNSUPPORTED, "dissipative stabilisation with local time steps at p = " +
                                            std::to_string(a - 1) + ", q = " + std::to_string(q));
    }
  }
  ++m->epoch;
  const size_t bytes = sizeof(double) * Mesh::kDissWords * m->ne, bytes32 = sizeof(float) * Mesh::kDissWords * m->ne;
  if (c == 0.0) {
    if (m->d_diss) {
      dev_free(m->ctx, m->d_diss, bytes);
      dev_free(m->ctx, m->d_diss32, bytes32);
      m->device_bytes -= bytes + bytes32;
    }
    m->d_diss = nullptr;
    m->d_diss32 = nullptr;
    m->c_diss = 0.0;
    return STDG_OK;
  }
  std::vector<double> h((size_t)Mesh::kDissWords * m->ne, 0.0);
  for (int64_t e = 0; e < m->ne; ++e) {
    double* o = h.data() + (size_t)Mesh::kDissWords * e;
    const ElemMetric& M = m->metric[e];
    const double ze = std::sqrt(M.mu / M.eps), zh = std::sqrt(M.eps / M.mu);
    for (int g = 0; g < 6; ++g) {
      const int k = m->info[e].nb[g];
      if (k < 0) {
        o[g] = c / ze;
        o[6 + g] = 0.0;
      } else {
        const ElemMetric& N = m->metric[k];
        o[g] = c / (0.5 * (ze + std::sqrt(N.mu / N.eps)));
        o[6 + g] = c / (0.5 * (zh + std::sqrt(N.eps / N.mu)));
      }
    }
    const double* X = m->verts.data() + 24 * e;
    double d[3][3];  // d[axis] = dF / dx-hat_axis (constant)
    for (int ax = 0; ax < 3; ++ax)
      for (int k = 0; k < 3; ++k) d[ax][k] = X[3 * (1 << ax) + k] - X[k];
    for (int al = 0; al < 3; ++al) {
      const double* ta = d[(al + 1) % 3];
      const double* tb = d[(al + 2) % 3];
      const double aa = ta[0] * ta[0] + ta[1] * ta[1] + ta[2] * ta[2];
      const double bb = tb[0] * tb[0] + tb[1] * tb[1] + tb[2] * tb[2];
      const double ab = ta[0] * tb[0] + ta[1] * tb[1] + ta[2] * tb[2];
      const double cx = ta[1] * tb[2] - ta[2] * tb[1], cy = ta[2] * tb[0] - ta[0] * tb[2],
                   cz = ta[0] * tb[1] - ta[1] * tb[0];
      const double area = std::sqrt(cx * cx + cy * cy + cz * cz);
      o[12 + 3 * al + 0] = bb / area;
      o[12 + 3 * al + 1] = aa / area;
      o[12 + 3 * al + 2] = -ab / area;
    }
  }
  if (!m->d_diss) {
    int rc = dev_alloc(m->ctx, (void**)&m->d_diss, bytes);
    if (rc != STDG_OK) return rc;
    rc = dev_alloc(m->ctx, (void**)&m->d_diss32, bytes32);
    if (rc != STDG_OK) {
      dev_free(m->ctx, m->d_diss, bytes);
      m->d_diss = nullptr;
      return rc;
    }
    m->device_bytes += bytes + bytes32;
  }
  std::vector<float> h32(h.begin(), h.end());
  STDG_HIP(hipMemcpy(m->d_diss, h.data(), bytes, hipMemcpyHostToDevice));
  STDG_HIP(hipMemcpy(m->d_diss32, h32.data(), bytes32, hipMemcpyHostToDevice));
  m->c_diss = c;
  return STDG_OK;
}

int build_mesh(Ctx* ctx, const stdg_mesh_desc* d, Mesh* m) {
  m->ctx = ctx;
  int rc = build_mesh_host(d, m);
  if (rc != STDG_OK) return rc;
  return upload_mesh(ctx, m);
}

void release_mesh(Mesh* m) {
  Ctx* ctx = m->ctx;
  release_cached_solver(m);
  for (int k = 0; k < Mesh::kAux; ++k) {
    if (m->aux[k]) (void)hipStreamDestroy(m->aux[k]);
    if (m->join_ev[k]) (void)hipEventDestroy(m->join_ev[k]);
    m->aux[k] = nullptr;
    m->join_ev[k] = nullptr;
  }
  if (m->fork_ev) (void)hipEventDestroy(m->fork_ev);
  m->fork_ev = nullptr;
  if (m->d_info) dev_free(ctx, m->d_info, sizeof(ElemInfo) * m->ne);
  if (m->d_metric) dev_free(ctx, m->d_metric, sizeof(ElemMetric) * m->ne);
  if (m->d_verts) dev_free(ctx, m->d_verts, sizeof(double) * 24 * m->ne);
  if (m->d_qt64) dev_free(ctx, m->d_qt64, sizeof(QTables<double>) * (kMaxA + 1));
  if (m->d_qt32) dev_free(ctx, m->d_qt32, sizeof(QTables<float>) * (kMaxA + 1));
  m->d_qt64 = m->d_qt32 = nullptr;
  if (m->d_hang) dev_free(ctx, m->d_hang, sizeof(HangRec) * m->hang.size());
  if (m->d_hs64) dev_free(ctx, m->d_hs64, sizeof(double) * 2 * kMaxA * kMaxA);
  if (m->d_hs32) dev_free(ctx, m->d_hs32, sizeof(float) * 2 * kMaxA * kMaxA);
  m->d_hang = nullptr;
  m->d_hs64 = m->d_hs32 = nullptr;
  if (m->d_lt) dev_free(ctx, m->d_lt, sizeof(LTRec) * m->lt.size());
  if (m->d_lt_work) dev_free(ctx, m->d_lt_work, sizeof(int32_t) * m->lt_work.size());
  m->d_lt_work = nullptr;
  if (m->d_ltb64) dev_free(ctx, m->d_ltb64, sizeof(double) * m->lt_bank.size());
  if (m->d_ltb32) dev_free(ctx, m->d_ltb32, sizeof(float) * m->lt_bank.size());
  m->d_lt = nullptr;
  m->d_ltb64 = m->d_ltb32 = nullptr;
  if (m->d_fr64) dev_free(ctx, m->d_fr64, sizeof(FaceRule<double>) * (kMaxFaceQ + 1));
  if (m->d_fr32) dev_free(ctx, m->d_fr32, sizeof(FaceRule<float>) * (kMaxFaceQ + 1));
  m->d_fr64 = m->d_fr32 = nullptr;
  for (auto& g : m->groups)
    if (g.d_list && ctx) dev_free(ctx, g.d_list, sizeof(int32_t) * g.count);
  if (m->d_scratch) dev_free(ctx, m->d_scratch, m->scratch_bytes);
  if (m->d_state_off) dev_free(ctx, m->d_state_off, sizeof(int64_t) * (m->ne + 1));
  if (m->d_diss) dev_free(ctx, m->d_diss, sizeof(double) * Mesh::kDissWords * m->ne);
  if (m->d_diss32) dev_free(ctx, m->d_diss32, sizeof(float) * Mesh::kDissWords * m->ne);
  m->d_diss = nullptr;
  m->d_diss32 = nullptr;
  m->c_diss = 0.0;
  m->d_state_off = nullptr;
  m->d_info = nullptr;
  m->d_metric = nullptr;
  m->d_verts = nullptr;
  m->groups.clear();
  m->d_scratch = nullptr;
}

}  // namespace stdg
