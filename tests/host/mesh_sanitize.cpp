// Host-only harness for the mesh builder and the 1D tables, built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitize.py
// (no device code, no GPU): valid lattices in every orientation, a 2:1
// hanging face (accepted) and a face split into cells that are not its
// quarters (refused), and invalid inputs that must be refused without
// touching memory they do not own.
#include <array>
#include <cmath>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../paper_1307_5310_amd/csrc/internal.h"

// the runtime pieces mesh.cpp and tables.cpp use, without a device
namespace stdg {
static std::string g_err;
void set_error(const std::string& m) { g_err = m; }
int fail(int status, const std::string& m) { g_err = m; return status; }
int hip_fail(hipError_t, const char* what) { g_err = what; return STDG_E_DEVICE; }
int dev_alloc(Ctx*, void**, size_t) { return STDG_E_DEVICE; }
void dev_free(Ctx*, void*, size_t) {}
void release_cached_solver(Mesh*) {}
}  // namespace stdg

struct Built {
  std::vector<double> v;
  std::vector<int64_t> h;
  int64_t ne = 0;
};

static Built lattice(int nx, int ny, int nz, unsigned seed, bool rotate) {
  Built b;
  auto id = [&](int i, int j, int k) { return (int64_t)i + (nx + 1) * ((int64_t)j + (ny + 1) * k); };
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        b.v.push_back(i * 0.5);
        b.v.push_back(j * 0.25 + 0.05 * i);
        b.v.push_back(k * 0.75);
      }
  // the 24 rotations of the cube as corner permutations
  std::vector<std::array<int, 8>> rots;
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (auto& pm : perms)
    for (int sg = 0; sg < 8; ++sg) {
      int R[3][3] = {{0}};
      for (int r = 0; r < 3; ++r) R[r][pm[r]] = (sg >> r) & 1 ? -1 : 1;
      const int det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) - R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
                      R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
      if (det != 1) continue;
      std::array<int, 8> p{};
      for (int v = 0; v < 8; ++v) {
        int s[3], o = 0;
        for (int d = 0; d < 3; ++d) s[d] = 2 * ((v >> d) & 1) - 1;
        for (int r = 0; r < 3; ++r) {
          int t = R[r][0] * s[0] + R[r][1] * s[1] + R[r][2] * s[2];
          o |= ((t + 1) / 2) << r;
        }
        p[v] = o;
      }
      rots.push_back(p);
    }
  unsigned st = seed;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t c[8];
        for (int v = 0; v < 8; ++v) c[v] = id(i + (v & 1), j + ((v >> 1) & 1), k + ((v >> 2) & 1));
        st = st * 1103515245u + 12345u;
        const auto& p = rots[rotate ? (st >> 8) % rots.size() : 0];
        for (int v = 0; v < 8; ++v) b.h.push_back(c[p[v]]);
        ++b.ne;
      }
  return b;
}

static int build(const Built& b, int p = 2, int q = 2, double eps = 1.0, int64_t* hanging = nullptr,
                 const std::vector<int32_t>* nsub = nullptr, stdg::Mesh* keep = nullptr) {
  std::vector<int32_t> pp(b.ne, p), qq(b.ne, q);
  std::vector<double> e(b.ne, eps), mu(b.ne, 1.0);
  stdg_mesh_desc d{(int64_t)(b.v.size() / 3), b.v.data(), b.ne, b.h.data(), pp.data(), qq.data(), e.data(), mu.data(),
                   nsub ? nsub->data() : nullptr};
  stdg::Mesh m;
  stdg::Mesh& mm = keep ? *keep : m;
  const int rc = stdg::build_mesh_host(&d, &mm);
  if (hanging) *hanging = mm.n_hanging_faces;
  return rc;
}

int main() {
  int bad = 0;
  auto expect = [&](const char* what, int got, int want) {
    if (got != want) {
      std::printf("FAIL %s: status %d, expected %d (%s)\n", what, got, want, stdg::g_err.c_str());
      ++bad;
    }
  };
  expect("canonical lattice", build(lattice(4, 3, 2, 1, false)), STDG_OK);
  for (unsigned s = 1; s <= 4; ++s) expect("rotated lattice", build(lattice(3, 3, 3, s, true)), STDG_OK);
  {
    Built b = lattice(2, 2, 2, 5, true);
    b.h[8 * 3 + 2] = (int64_t)(b.v.size() / 3) + 7;  // vertex id out of range
    expect("vertex id out of range", build(b), STDG_E_ARG);
  }
  {
    Built b = lattice(2, 1, 1, 6, false);
    b.v[4] = std::nan("");
    expect("non-finite coordinate", build(b), STDG_E_ARG);
  }
  {
    Built b = lattice(2, 1, 1, 7, false);
    for (int v = 0; v < 8; ++v) b.h[8 + v] = b.h[v];  // element 1 = element 0: coincident elements
    expect("duplicate element", build(b), STDG_E_ARG);
  }
  {
    Built b = lattice(1, 1, 1, 8, false);
    std::swap(b.h[0], b.h[1]);  // inverted element
    expect("inverted element", build(b), STDG_E_ARG);
  }
  expect("degree out of range", build(lattice(1, 1, 1, 9, false), 9, 1), STDG_E_ARG);
  expect("eps <= 0", build(lattice(1, 1, 1, 9, false), 2, 1, 0.0), STDG_E_ARG);
  {
    // a unit cube next to four half cubes: split face
    Built b;
    std::map<std::array<long, 3>, int64_t> idx;
    auto vid = [&](double x, double y, double z) {
      std::array<long, 3> k{std::lround(x * 1e6), std::lround(y * 1e6), std::lround(z * 1e6)};
      auto it = idx.find(k);
      if (it != idx.end()) return it->second;
      const int64_t n = (int64_t)(b.v.size() / 3);
      idx[k] = n;
      b.v.insert(b.v.end(), {x, y, z});
      return n;
    };
    auto hexa = [&](double x0, double y0, double z0, double h) {
      for (int v = 0; v < 8; ++v) b.h.push_back(vid(x0 + h * (v & 1), y0 + h * ((v >> 1) & 1), z0 + h * ((v >> 2) & 1)));
      ++b.ne;
    };
    hexa(0, 0, 0, 1);
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k) hexa(1, 0.5 * j, 0.5 * k, 0.5);
    int64_t nh = -1;
    expect("2:1 hanging face", build(b, 2, 2, 1.0, &nh), STDG_OK);
    std::vector<int32_t> ns(b.ne, 1);
    ns[2] = 2;
    expect("local time steps with hanging faces", build(b, 2, 2, 1.0, nullptr, &ns), STDG_E_UNSUPPORTED);
    if (nh != 1) {
      std::printf("FAIL 2:1 hanging face: %lld hanging faces recorded, expected 1\n", (long long)nh);
      ++bad;
    }
    // the same cells with the centre vertex of the split face duplicated for
    // one small cell (unshared vertex ids at one position): its face is not a
    // quarter by vertex ids, yet the small faces' centroids sit at the coarse
    // face's quarter points: refused rather than taken for walls
    Built c = b;
    int64_t centre = -1;
    for (size_t i = 0; i + 2 < c.v.size(); i += 3)
      if (std::fabs(c.v[i] - 1.0) < 1e-9 && std::fabs(c.v[i + 1] - 0.5) < 1e-9 && std::fabs(c.v[i + 2] - 0.5) < 1e-9)
        centre = (int64_t)(i / 3);
    const int64_t dup = (int64_t)(c.v.size() / 3);
    c.v.insert(c.v.end(), {1.0, 0.5, 0.5});
    for (int v = 0; v < 8; ++v)
      if (c.h[8 * 1 + v] == centre) c.h[8 * 1 + v] = dup;
    expect("split face, not quarters", build(c), STDG_E_UNSUPPORTED);
  }
  // local time steps: sub-intervals per element; the rows of elements with
  // several, and of their face neighbours, leave the kernel groups
  {
    Built b = lattice(3, 3, 3, 11, true);
    std::vector<int32_t> ns(b.ne, 1);
    ns[0] = 2;
    ns[13] = 4;
    ns[26] = 8;
    stdg::Mesh m;
    expect("local time steps", build(b, 2, 2, 1.0, nullptr, &ns, &m), STDG_OK);
    int64_t grouped = 0, local = 0, want = 0;
    for (const auto& g : m.groups) grouped += g.count;
    for (int64_t e = 0; e < b.ne; ++e) {
      bool l = ns[e] > 1;
      for (int f = 0; f < 6; ++f)
        if (m.info[e].nb[f] >= 0 && ns[m.info[e].nb[f]] > 1) l = true;
      want += l;
      local += (m.info[e].flags & stdg::kLocalTime) != 0;
    }
    if (local != want || (int64_t)m.lt.size() != want || grouped + want != b.ne) {
      std::printf("FAIL local time rows: %lld flagged, %zu records, %lld grouped, expected %lld local of %lld\n",
                  (long long)local, m.lt.size(), (long long)grouped, (long long)want, (long long)b.ne);
      ++bad;
    }
    int64_t unk = 0;
    for (int64_t e = 0; e < b.ne; ++e) unk += 6 * 2 * ns[e] * 27;
    if (m.unk_off.back() != unk || m.trial_off.back() != unk + 6 * 27 * b.ne) {
      std::printf("FAIL local time offsets\n");
      ++bad;
    }
    for (int bad_n : {3, 16, 0}) {
      std::vector<int32_t> nb(b.ne, 1);
      nb[5] = bad_n;
      expect("sub-intervals not a power of two in 1..8", build(b, 2, 2, 1.0, nullptr, &nb), STDG_E_ARG);
    }
    std::vector<int32_t> big(b.ne, 1);
    big[5] = 8;
    expect("sub-intervals times q > 24", build(b, 2, 4, 1.0, nullptr, &big), STDG_E_ARG);
    Built t = b;
    t.v[3 * (1 + 4 * (1 + 4 * 1)) + 2] += 0.05;  // an interior vertex moved: trilinear elements
    expect("local time steps on trilinear elements", build(t, 2, 2, 1.0, nullptr, &ns), STDG_E_UNSUPPORTED);
  }
  // tables
  for (int n = 1; n <= 16; ++n) {
    double x[16], w[16];
    stdg::gauss_rule01(n, x, w);
    double s = 0;
    for (int i = 0; i < n; ++i) s += w[i];
    if (std::fabs(s - 1.0) > 1e-13) { std::printf("FAIL gauss weights n=%d\n", n); ++bad; }
  }
  for (int a = 1; a <= stdg::kMaxA; ++a) {
    stdg::QTables<double> t64;
    stdg::QTables<float> t32;
    stdg::fill_qtables_f64(a, &t64);
    stdg::fill_qtables_f32(a, &t32);
  }
  stdg::Tables<double> T64;
  stdg::Tables<float> T32;
  stdg::fill_tables_f64(&T64);
  stdg::fill_tables_f32(&T32);
  std::printf(bad ? "harness: %d failures\n" : "harness: all cases as expected\n", bad);
  return bad ? 1 : 0;
}
