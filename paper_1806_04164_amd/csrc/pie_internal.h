// Internal structures of the PIE / MLFMA library (host side).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pie.h"

namespace pie {

constexpr double kPi = 3.14159265358979323846;
constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr double kEps0 = 1.0 / (kMu0 * kC0 * kC0);
constexpr int kNumOffsets = 316;  // far offsets in [-3,3]^3 with max|.| >= 2
constexpr int kComp = 5;          // pattern components Jx, Jy, Jz, sigma, u

void set_error(const std::string& msg);

struct Mesh {
  int64_t nv = 0, nt = 0, ne = 0;
  std::vector<double> V;        // [nv][3]
  std::vector<int32_t> T;       // [nt][3]
  std::vector<int32_t> edge;    // [ne][2] (a < b)
  std::vector<int32_t> etri;    // [ne][2] (T+, T-)
  std::vector<int32_t> efree;   // [ne][2] (p+, p-)
  std::vector<double> elen;     // [ne]
  std::vector<double> area;     // [nt]
  std::vector<double> normal;   // [nt][3]
  std::vector<double> centroid; // [nt][3]
  int64_t nboundary = 0;
};

struct Level {
  int l = 0;
  int64_t nb = 0;
  std::vector<int64_t> code;    // Morton codes (sorted)
  std::vector<int64_t> coords;  // [nb][3]
  std::vector<int64_t> parent;  // [nb]
  std::vector<int64_t> child_ptr;  // [nb+1] into level l+1 (l < L)
  std::vector<int64_t> il_ptr, il_src, il_off;  // l >= 3
};

struct Tree {
  int L = 0;
  int64_t N = 0;
  double origin[3] = {0, 0, 0};
  double side = 0;
  std::vector<Level> lev;        // index l (0 unused)
  std::vector<int64_t> box_of;   // [N] finest box of canonical unknown
  std::vector<int64_t> perm;     // [N] canonical index at box-order slot
  std::vector<int64_t> box_ptr;  // [nbL+1]
  std::vector<int64_t> near_ptr, near_idx;
  const Mesh* mesh = nullptr;
};

pie_status build_mesh(const double* V, int64_t nv, const int32_t* T, int64_t nt, Mesh& m);
pie_status build_tree(const Mesh& m, int L, Tree& t);
// Icosphere of radius `radius` with 20 * 4^subdiv triangles (host, bit-reproducible).
pie_status icosphere(int subdiv, double radius, double jitter, uint64_t seed, std::vector<double>& V,
                     std::vector<int32_t>& T);
int64_t morton3(int64_t x, int64_t y, int64_t z);
int offset_id(int64_t dx, int64_t dy, int64_t dz);

// --------------------------------------------------------------- tables --
// Gauss-Legendre nodes/weights on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// k * s^t * h_t^(1)(k w) for t = 0..tau (re, im interleaved).
void scaled_hankel(double k, double s, double w, int tau, std::vector<double>& out);

}  // namespace pie
