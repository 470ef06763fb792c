// Mesh tables (RWG and pulse discretisation, Section 2) and cubic-box
// clustering with one-box-buffer near and interaction lists (Section 3).
// Host C++, integer and FP64.  Built with -ffp-contract=off so that the box
// assignment of every basis function is reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <unordered_map>
#include <limits>

#include "pie_internal.h"

namespace pie {

pie_status build_mesh(const double* V, int64_t nv, const int32_t* T, int64_t nt, Mesh& m) {
  if (!V || !T || nv < 3 || nt < 1) {
    set_error("mesh: null array or empty mesh");
    return PIE_ERR_ARG;
  }
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(V[i])) {
      set_error("mesh: non-finite vertex coordinate");
      return PIE_ERR_NONFINITE;
    }
  for (int64_t i = 0; i < 3 * nt; ++i)
    if (T[i] < 0 || T[i] >= nv) {
      set_error("mesh: triangle vertex index out of range");
      return PIE_ERR_ARG;
    }
  m.nv = nv;
  m.nt = nt;
  m.V.assign(V, V + 3 * nv);
  m.T.assign(T, T + 3 * nt);
  m.area.resize(nt);
  m.normal.resize(3 * nt);
  m.centroid.resize(3 * nt);
  for (int64_t t = 0; t < nt; ++t) {
    const double* a = &V[3 * T[3 * t + 0]];
    const double* b = &V[3 * T[3 * t + 1]];
    const double* c = &V[3 * T[3 * t + 2]];
    double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(len > 0.0)) {
      set_error("mesh: degenerate triangle " + std::to_string(t));
      return PIE_ERR_MESH;
    }
    m.area[t] = 0.5 * len;
    for (int d = 0; d < 3; ++d) {
      m.normal[3 * t + d] = n[d] / len;
      m.centroid[3 * t + d] = ((a[d] + b[d]) + c[d]) / 3.0;
    }
  }
  // Half-edges (from, to, triangle, opposite vertex), grouped by the
  // undirected edge (min, max); within a group the a->b traversal first.
  struct HalfEdge {
    int32_t lo, hi, tri, opp;
    bool fwd;
  };
  std::vector<HalfEdge> he(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      int32_t f = T[3 * t + k], to = T[3 * t + (k + 1) % 3], o = T[3 * t + (k + 2) % 3];
      he[3 * t + k] = {std::min(f, to), std::max(f, to), (int32_t)t, o, f < to};
    }
  std::sort(he.begin(), he.end(), [](const HalfEdge& x, const HalfEdge& y) {
    if (x.lo != y.lo) return x.lo < y.lo;
    if (x.hi != y.hi) return x.hi < y.hi;
    if (x.fwd != y.fwd) return x.fwd;  // forward (a->b) first
    return x.tri < y.tri;
  });
  m.edge.clear();
  m.etri.clear();
  m.efree.clear();
  m.elen.clear();
  m.nboundary = 0;
  size_t i = 0;
  while (i < he.size()) {
    size_t j = i;
    while (j < he.size() && he[j].lo == he[i].lo && he[j].hi == he[i].hi) ++j;
    size_t cnt = j - i;
    if (cnt > 2) {
      set_error("mesh: non-manifold edge shared by more than two triangles");
      return PIE_ERR_MESH;
    }
    if (cnt == 2) {
      if (!he[i].fwd || he[i + 1].fwd) {
        set_error("mesh: inconsistently oriented triangles");
        return PIE_ERR_MESH;
      }
      m.edge.push_back(he[i].lo);
      m.edge.push_back(he[i].hi);
      m.etri.push_back(he[i].tri);
      m.etri.push_back(he[i + 1].tri);
      m.efree.push_back(he[i].opp);
      m.efree.push_back(he[i + 1].opp);
      const double* a = &V[3 * he[i].lo];
      const double* b = &V[3 * he[i].hi];
      double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
      m.elen.push_back(std::sqrt(dx * dx + dy * dy + dz * dz));
    } else {
      ++m.nboundary;
    }
    i = j;
  }
  m.ne = (int64_t)m.elen.size();
  return PIE_OK;
}

int64_t morton3(int64_t x, int64_t y, int64_t z) {
  int64_t c = 0;
  for (int b = 0; b < 21; ++b) {
    c |= ((x >> b) & 1) << (3 * b);
    c |= ((y >> b) & 1) << (3 * b + 1);
    c |= ((z >> b) & 1) << (3 * b + 2);
  }
  return c;
}

int offset_id(int64_t dx, int64_t dy, int64_t dz) {
  // lexicographic rank among vectors of [-3,3]^3 with max|.| >= 2
  int id = 0;
  for (int a = -3; a <= 3; ++a)
    for (int b = -3; b <= 3; ++b)
      for (int c = -3; c <= 3; ++c) {
        if (std::max({std::abs(a), std::abs(b), std::abs(c)}) < 2) continue;
        if (a == dx && b == dy && c == dz) return id;
        ++id;
      }
  return -1;
}

static int64_t find_code(const std::vector<int64_t>& codes, int64_t c) {
  auto it = std::lower_bound(codes.begin(), codes.end(), c);
  if (it == codes.end() || *it != c) return -1;
  return it - codes.begin();
}

pie_status build_tree(const Mesh& m, int L, Tree& t) {
  if (L < 3 || L > 21) {
    set_error("tree: levels must be in [3, 21]");
    return PIE_ERR_ARG;
  }
  t.L = L;
  t.mesh = &m;
  const int64_t N = m.ne + m.nt;
  t.N = N;
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) lo[d] = hi[d] = m.V[d];
  for (int64_t v = 0; v < m.nv; ++v)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], m.V[3 * v + d]);
      hi[d] = std::max(hi[d], m.V[3 * v + d]);
    }
  double side = 0.0;
  double centre[3];
  for (int d = 0; d < 3; ++d) {
    centre[d] = (lo[d] + hi[d]) / 2.0;
    side = std::max(side, hi[d] - lo[d]);
  }
  if (!(side > 0.0)) {
    set_error("tree: zero-size object");
    return PIE_ERR_MESH;
  }
  t.side = side;
  for (int d = 0; d < 3; ++d) t.origin[d] = centre[d] - side / 2.0;
  const int64_t nL = int64_t(1) << (L - 1);
  std::vector<int64_t> ic(3 * N);
  for (int64_t u = 0; u < N; ++u) {
    double p[3];
    if (u < m.ne) {
      const double* a = &m.V[3 * m.edge[2 * u]];
      const double* b = &m.V[3 * m.edge[2 * u + 1]];
      for (int d = 0; d < 3; ++d) p[d] = (a[d] + b[d]) * 0.5;
    } else {
      const int32_t* tv = &m.T[3 * (u - m.ne)];
      for (int d = 0; d < 3; ++d)
        p[d] = ((m.V[3 * tv[0] + d] + m.V[3 * tv[1] + d]) + m.V[3 * tv[2] + d]) / 3.0;
    }
    for (int d = 0; d < 3; ++d) {
      double tt = (p[d] - t.origin[d]) / side;
      double f = std::floor(tt * (double)nL);
      int64_t i = (int64_t)f;
      if (f < 0.0) i = 0;
      if (i > nL - 1) i = nL - 1;
      ic[3 * u + d] = i;
    }
  }
  std::vector<int64_t> codeL(N);
  for (int64_t u = 0; u < N; ++u) codeL[u] = morton3(ic[3 * u], ic[3 * u + 1], ic[3 * u + 2]);
  t.perm.resize(N);
  std::iota(t.perm.begin(), t.perm.end(), 0);
  std::sort(t.perm.begin(), t.perm.end(), [&](int64_t a, int64_t b) {
    if (codeL[a] != codeL[b]) return codeL[a] < codeL[b];
    int ka = a >= m.ne, kb = b >= m.ne;
    if (ka != kb) return ka < kb;
    return a < b;
  });
  t.lev.assign(L + 1, Level());
  for (int l = 1; l <= L; ++l) {
    Level& lv = t.lev[l];
    lv.l = l;
    int sh = L - l;
    std::vector<int64_t> codes(N);
    for (int64_t u = 0; u < N; ++u)
      codes[u] = morton3(ic[3 * u] >> sh, ic[3 * u + 1] >> sh, ic[3 * u + 2] >> sh);
    std::sort(codes.begin(), codes.end());
    codes.erase(std::unique(codes.begin(), codes.end()), codes.end());
    lv.code = codes;
    lv.nb = (int64_t)codes.size();
    lv.coords.resize(3 * lv.nb);
    for (int64_t b = 0; b < lv.nb; ++b) {
      int64_t x = 0, y = 0, z = 0, c = codes[b];
      for (int k = 0; k < 21; ++k) {
        x |= ((c >> (3 * k)) & 1) << k;
        y |= ((c >> (3 * k + 1)) & 1) << k;
        z |= ((c >> (3 * k + 2)) & 1) << k;
      }
      lv.coords[3 * b] = x;
      lv.coords[3 * b + 1] = y;
      lv.coords[3 * b + 2] = z;
    }
  }
  for (int l = 1; l <= L; ++l) {
    Level& lv = t.lev[l];
    lv.parent.assign(lv.nb, -1);
    if (l > 1)
      for (int64_t b = 0; b < lv.nb; ++b) lv.parent[b] = find_code(t.lev[l - 1].code, lv.code[b] >> 3);
    if (l < L) {
      const Level& ch = t.lev[l + 1];
      lv.child_ptr.assign(lv.nb + 1, 0);
      for (int64_t c = 0; c < ch.nb; ++c) {
        int64_t p = find_code(lv.code, ch.code[c] >> 3);
        lv.child_ptr[p + 1]++;
      }
      for (int64_t b = 0; b < lv.nb; ++b) lv.child_ptr[b + 1] += lv.child_ptr[b];
    }
  }
  const Level& fl = t.lev[L];
  t.box_of.resize(N);
  for (int64_t u = 0; u < N; ++u) t.box_of[u] = find_code(fl.code, codeL[u]);
  t.box_ptr.assign(fl.nb + 1, 0);
  for (int64_t u = 0; u < N; ++u) t.box_ptr[t.box_of[u] + 1]++;
  for (int64_t b = 0; b < fl.nb; ++b) t.box_ptr[b + 1] += t.box_ptr[b];
  // near lists (ascending box index)
  t.near_ptr.assign(1, 0);
  t.near_idx.clear();
  for (int64_t b = 0; b < fl.nb; ++b) {
    std::vector<int64_t> nb;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          int64_t x = fl.coords[3 * b] + dx, y = fl.coords[3 * b + 1] + dy, z = fl.coords[3 * b + 2] + dz;
          if (x < 0 || y < 0 || z < 0 || x >= nL || y >= nL || z >= nL) continue;
          int64_t j = find_code(fl.code, morton3(x, y, z));
          if (j >= 0) nb.push_back(j);
        }
    std::sort(nb.begin(), nb.end());
    t.near_idx.insert(t.near_idx.end(), nb.begin(), nb.end());
    t.near_ptr.push_back((int64_t)t.near_idx.size());
  }
  // interaction lists: children of the parent's near boxes that are not near
  for (int l = 3; l <= L; ++l) {
    Level& lv = t.lev[l];
    const Level& up = t.lev[l - 1];
    const int64_t nl = int64_t(1) << (l - 2);  // boxes per side at level l-1
    lv.il_ptr.assign(1, 0);
    lv.il_src.clear();
    lv.il_off.clear();
    for (int64_t b = 0; b < lv.nb; ++b) {
      int64_t p = lv.parent[b];
      std::vector<std::pair<int64_t, int>> cand;
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            int64_t x = up.coords[3 * p] + dx, y = up.coords[3 * p + 1] + dy, z = up.coords[3 * p + 2] + dz;
            if (x < 0 || y < 0 || z < 0 || x >= nl || y >= nl || z >= nl) continue;
            int64_t q = find_code(up.code, morton3(x, y, z));
            if (q < 0) continue;
            for (int64_t c = up.child_ptr[q]; c < up.child_ptr[q + 1]; ++c) {
              int64_t ddx = lv.coords[3 * b] - lv.coords[3 * c];
              int64_t ddy = lv.coords[3 * b + 1] - lv.coords[3 * c + 1];
              int64_t ddz = lv.coords[3 * b + 2] - lv.coords[3 * c + 2];
              if (std::max({std::llabs(ddx), std::llabs(ddy), std::llabs(ddz)}) < 2) continue;
              cand.push_back({c, offset_id(ddx, ddy, ddz)});
            }
          }
      std::sort(cand.begin(), cand.end());
      for (auto& cc : cand) {
        lv.il_src.push_back(cc.first);
        lv.il_off.push_back(cc.second);
      }
      lv.il_ptr.push_back((int64_t)lv.il_src.size());
    }
  }
  return PIE_OK;
}


// ------------------------------------------------------------ icosphere --
// The sphere meshes of the Section 4 experiments, generated here so that a
// caller can build a workload without its own mesher.  Built with
// -ffp-contract=off; every coordinate is formed by the operation sequence
// written below (norms as ((x*x + y*y) + z*z), midpoints as 0.5 * (a + b)
// then divided by their norm), so that results are reproducible bit for bit
// on any IEEE host.
namespace {

double norm3(double x, double y, double z) { return std::sqrt((x * x + y * y) + z * z); }

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): draw n (n = 0, 1, ...) of
// the stream started at seed is mix(seed + (n + 1) * gamma).
uint64_t splitmix(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

pie_status icosphere(int subdiv, double radius, double jitter, uint64_t seed, std::vector<double>& V,
                     std::vector<int32_t>& T) {
  if (subdiv < 0 || subdiv > 10 || !(radius > 0.0) || !std::isfinite(radius) || !(jitter >= 0.0) ||
      !(jitter < 0.5)) {
    set_error("icosphere: need 0 <= subdiv <= 10, radius > 0 and 0 <= jitter < 0.5");
    return PIE_ERR_ARG;
  }
  // the 12 vertices of the regular icosahedron: (0, a, b), (a, b, 0),
  // (b, 0, a) for a = -1, 1 and b = -g, g (g the golden ratio), on the unit
  // sphere
  const double g = (1.0 + std::pow(5.0, 0.5)) / 2.0;
  V.clear();
  for (double a : {-1.0, 1.0})
    for (double b : {-g, g}) {
      const double p[3][3] = {{0.0, a, b}, {a, b, 0.0}, {b, 0.0, a}};
      for (const auto& q : p) {
        const double n = norm3(q[0], q[1], q[2]);
        V.insert(V.end(), {q[0] / n, q[1] / n, q[2] / n});
      }
    }
  // faces: triples of mutually adjacent vertices (shortest chord), i < j < k,
  // oriented counter-clockwise seen from outside
  auto dist = [&](int i, int j) {
    return norm3(V[3 * i] - V[3 * j], V[3 * i + 1] - V[3 * j + 1], V[3 * i + 2] - V[3 * j + 2]);
  };
  double e = 1e300;
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < 12; ++j)
      if (i != j) e = std::min(e, dist(i, j));
  auto adj = [&](int i, int j) { return std::abs(dist(i, j) - e) < 1e-9; };
  std::vector<int64_t> F;
  for (int i = 0; i < 12; ++i)
    for (int j = i + 1; j < 12; ++j) {
      if (!adj(i, j)) continue;
      for (int k = j + 1; k < 12; ++k) {
        if (!adj(i, k) || !adj(j, k)) continue;
        const double* a = &V[3 * i];
        const double* b = &V[3 * j];
        const double* c = &V[3 * k];
        const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        const double d = n[0] * (a[0] + b[0] + c[0]) + n[1] * (a[1] + b[1] + c[1]) + n[2] * (a[2] + b[2] + c[2]);
        if (d < 0.0)
          F.insert(F.end(), {i, k, j});
        else
          F.insert(F.end(), {i, j, k});
      }
    }
  if (F.size() != 60) {
    set_error("icosphere: icosahedron construction failed");
    return PIE_ERR_MESH;
  }
  // subdivision: every face into four; a new vertex (the normalised
  // midpoint) is appended when an edge is first met, walking the faces in
  // order and each face's edges v0v1, v1v2, v2v0
  for (int s = 0; s < subdiv; ++s) {
    const int64_t nv = (int64_t)V.size() / 3, nf = (int64_t)F.size() / 3;
    std::unordered_map<int64_t, int64_t> mid;
    mid.reserve(2 * nf);
    std::vector<int64_t> NF;
    NF.reserve(12 * nf);
    int64_t next = nv;
    for (int64_t f = 0; f < nf; ++f) {
      int64_t m[3];
      for (int k = 0; k < 3; ++k) {
        const int64_t a = F[3 * f + k], b = F[3 * f + (k + 1) % 3];
        const int64_t lo = std::min(a, b), hi = std::max(a, b), key = lo * nv + hi;
        auto it = mid.find(key);
        if (it == mid.end()) {
          double p[3];
          for (int c = 0; c < 3; ++c) p[c] = 0.5 * (V[3 * lo + c] + V[3 * hi + c]);
          const double n = norm3(p[0], p[1], p[2]);
          V.insert(V.end(), {p[0] / n, p[1] / n, p[2] / n});
          it = mid.emplace(key, next++).first;
        }
        m[k] = it->second;  // m01, m12, m20
      }
      const int64_t v0 = F[3 * f], v1 = F[3 * f + 1], v2 = F[3 * f + 2];
      NF.insert(NF.end(), {v0, m[0], m[2], v1, m[1], m[0], v2, m[2], m[1], m[0], m[1], m[2]});
    }
    F.swap(NF);
  }
  for (double& c : V) c = c * radius;
  if (jitter > 0.0) {
    // vertex v moves by jitter * h_v * (2 u - 1) per coordinate, h_v the
    // shortest edge at v, u = draw 3 v + c of SplitMix64(seed) scaled to [0, 1)
    const int64_t nv = (int64_t)V.size() / 3;
    std::vector<double> h(nv, std::numeric_limits<double>::infinity());
    for (size_t f = 0; f < F.size(); f += 3)
      for (int k = 0; k < 3; ++k) {
        const int64_t a = F[f + k], b = F[f + (k + 1) % 3];
        const double L = norm3(V[3 * a] - V[3 * b], V[3 * a + 1] - V[3 * b + 1], V[3 * a + 2] - V[3 * b + 2]);
        h[a] = std::min(h[a], L);
        h[b] = std::min(h[b], L);
      }
    for (int64_t v = 0; v < nv; ++v)
      for (int c = 0; c < 3; ++c) {
        const double u = (double)(splitmix(seed, (uint64_t)(3 * v + c)) >> 11) * 0x1.0p-53;
        V[3 * v + c] = V[3 * v + c] + (jitter * h[v]) * (2.0 * u - 1.0);
      }
  }
  T.assign(F.begin(), F.end());
  return PIE_OK;
}

}  // namespace pie
