// Device data descriptors and small helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pie {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) {
  return cx<T>{r, i};
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) {
  return {s * a.re, s * a.im};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) {
  return {a.re, -a.im};
}
// a += b * c
template <typename T>
__device__ __forceinline__ void cfma(cx<T>& a, cx<T> b, cx<T> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}
// a += conj(b) * c
template <typename T>
__device__ __forceinline__ void cfma_conj(cx<T>& a, cx<T> b, cx<T> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(-b.im, c.re, a.im);
}

// Workgroup -> box index with consecutive boxes (Morton order, i.e. spatial
// neighbours) on the same XCD: workgroups are dispatched round-robin over
// the 8 XCDs, so workgroup w runs on XCD w % 8; box = (w % 8) * per + w / 8.
// The grid is 8 * per; returns -1 for the padding workgroups.
__device__ __forceinline__ int xcd_box(int w, int nb) {
  const int per = (nb + 7) >> 3;
  const int b = (w & 7) * per + (w >> 3);
  return b < nb ? b : -1;
}
__host__ __device__ __forceinline__ unsigned xcd_grid(int nb) { return 8u * (unsigned)((nb + 7) >> 3); }

// Geometry (FP64).
struct DevGeo {
  const double* V;    // [nv][3]
  const int32_t* T;   // [nt][3]
  const double* P;    // [nt][7][3] quadrature points
  const double* W;    // [nt][7] quadrature weights (area * rule weight)
  const double* C;    // [nt][3] centroids
  const double* Nrm;  // [nt][3] unit normals
  int32_t nt;
};

// Basis functions in box order (slot u); canonical index perm[u];
// RWG if perm[u] < ne.  Two halves per RWG (T+, T-): triangle, free vertex,
// vector scale +-l/(2A) and divergence +-l/A.  Pulses use tri[2u] only.
struct DevBasis {
  const int32_t* perm;
  const int32_t* tri;
  const int32_t* fv;
  const double* s;
  const double* d;
  int32_t N, ne;
};

// The scalar operator's sources per triangle t (canonical order): the RWG
// functions on its (up to three) edges and their divergence +-l/A on t, so
// that u_t = div J on t + w^2 eps0 x_A[t] = sum_k d[3t+k] x[e[3t+k]] + w^2 eps0
// x[ne + t]; e = -1 for an edge without an RWG function (open surfaces).
struct DevTriDiv {
  const int32_t* e;  // [nt][3]
  const double* d;   // [nt][3]
  int32_t nt, ne;
};

// Stored near-field blocks (a <= b, Morton box indices), row-major n_a x n_b,
// processed as row-panel tasks of at most one LDS panel each.
// One row panel [i0, i0 + nr) of a stored near block (a, b): 32 bytes, so a
// workgroup reads it with one load.
struct NearTaskDesc {
  int64_t off;   // entry offset of the panel in the stored blocks
  int32_t v0;    // first box-order unknown of box b (row sums read x there)
  int32_t nb;    // unknowns of box b = panel row length
  int32_t ua;    // box-order unknown of the panel's first row (column sums read x there)
  int32_t nr;    // rows in the panel
  int32_t prow;  // partial-sum slot of the panel's first row
  int32_t pcol;  // partial-sum slot of its column sums, -1 on a diagonal block
};
static_assert(sizeof(NearTaskDesc) == 32, "task descriptor is 8 dwords");

// One block-sparse near-field structure: either the RWG-RWG blocks (entries
// mu0 <f_m, int f_n g>, slots = the RWG functions in box order) or the
// triangle-triangle blocks (entries S_qp = <P_q, int P_p g>, slots = the
// triangles in box order).  Each box's slots are contiguous.
struct DevNear {
  int32_t kind;             // 0: RWG-RWG, 1: triangle-triangle
  int32_t nblk;
  const int32_t* blk_a;
  const int32_t* blk_b;
  const int64_t* blk_off;   // entry offset of each block
  const int32_t* prow;      // partial-sum slot of the block's rows
  int32_t ntask;
  const struct NearTaskDesc* tdesc;  // [ntask] one row panel per SpMM work unit
  const int32_t* pcol;      // task -> partial-sum slot of its column sums (a < b)
  // near boxes: a finest box's slots in runs of at most 128 (its box order)
  const int32_t* slot_ptr;  // [nv+1] slot ranges of the near boxes
  const int32_t* ubase;     // [nv] box-order unknown of each near box's first slot
  const int32_t* vptr;      // [nbL+1] near boxes of each finest box (slot run c = chunk c of 128)
  const int32_t* row_ptr;   // [nv+1] blocks whose a is the near box
  const int32_t* col_ptr;   // [nv+1] into col_blk
  const int32_t* col_blk;   // tasks of blocks (a < b) whose b is the near box
};

// One tree level.
struct DevLevel {
  int32_t nb;
  const double* centre;     // [nb][3]
  const int32_t* parent;    // [nb]
  const int32_t* octant;    // [nb] position in the parent (bit0 x, bit1 y, bit2 z)
  const int32_t* child_ptr; // [nb+1] into the next finer level
  const int32_t* il_ptr;    // [nb+1]
  const int32_t* il_src;
  const int32_t* il_off;
  int32_t nug;              // parent groups of the upward shift into this level
  const int32_t* ug_ptr;    // [nug+1] parent ranges; each group has <= SHIFT_GROUP children
  // batched translation by groups of at most TG_BOXES boxes of one parent
  // (siblings share most of their interaction-list sources): each group
  // lists the ascending union of its boxes' sources once, with the offset
  // index of every box that has the source in its list
  int32_t ntg;              // groups
  const int32_t* tg_box;    // [ntg+1] box ranges
  const int32_t* tg_ent;    // [ntg+1] ranges into te
  const int4* te;           // {source box, offset of box 0 | box 1 << 16, box 2 | box 3 << 16, 0};
                            //   offset 0xffff: the source is not in that box's list
};

// Inter-level shift tiling: sample rows per thread, boxes per workgroup.
constexpr int SQT = 8;
constexpr int SHIFT_GROUP = 12;
// Longest interaction list with a one-box buffer: 6^3 - 3^3 offsets.
constexpr int IL_MAX = 189;
// Translation offsets (max-norm 2 or 3 in box units).
constexpr int TRANSLATE_OFFSETS = 316;
// Batched translation: boxes per group, samples per workgroup (one per
// wavefront), columns per wavefront pass.
constexpr int TG_BOXES = 4;
constexpr int TG_Q = 4;
constexpr int TG_COLS = 64;

// (finest box, triangle) incidences: up to three RWG functions of the box
// that live on the triangle, and the triangle's pulse if the triangle belongs
// to the box (its home incidence: the scalar sources sigma and u of the
// triangle radiate and are received there).  Geometry is stored relative to
// the box centre C, so that a thread forms a quadrature point's source
// density or testing integral from independent loads only.
struct DevInc {
  const int32_t* ptr;   // [nbL+1] incidence range of each finest box
  const double* pw;     // [ninc][7][4] (r_i - C, quadrature weight W_i)
  const int32_t* xc;    // [ninc][4] canonical unknown of RWG slot k < 3 / of the pulse (k = 3), or -1
  const double* rs;     // [ninc][3] +-l/(2A)  (0 for an empty slot)
  const double* pv;     // [ninc][3][3] free vertex - C (0 for an empty slot)
  // per box-order unknown u and half h (a pulse uses h = 0 only)
  const int32_t* uj;    // [N][2] incidence index
  const double* us;     // [N][2] +-l/(2A)
  const double* upv;    // [N][2][3] free vertex - C
  const int32_t* uptr;  // [nbL+1] box-order unknown range of each finest box
  DevTriDiv td;         // divergence sources of the triangles
};

}  // namespace pie
