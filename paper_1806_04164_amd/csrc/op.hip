// Operator setup, MVM orchestration, GMRES and the C ABI.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstddef>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "pie_internal.h"

using pie::cx;

namespace pie {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

}  // namespace pie

struct pie_mesh {
  pie::Mesh m;
};
struct pie_tree {
  pie::Tree t;
};

struct pie_op {
  const pie::Mesh* mesh = nullptr;
  const pie::Tree* tree = nullptr;
  int device = 0;
  double freq = 0, omega = 0, k = 0, w2e = 0;
  int near_prec = 64, far_prec = 64, tau = 0, nth = 0, nph = 0, Q = 0;
  double xs = 0;
  int max_rhs = 1, rc = 1, L = 0, N = 0, ne = 0, nt = 0;
  int pw = 1;  // RHS columns per MVM pass (workspace width): min(max_rhs, kPassMax)
  int maxinc = 0;   // most (box, triangle) incidences of a finest box
  int maxjoin = 0;  // longest near-field join list of a finest box
  int lds_budget = 65536;  // dynamic LDS of the single-column aggregation and reception
  int nsplit = 1;  // aggregation incidence-loop split (fixed per operator: RHS-batch-independent order)
  // device geometry
  double *dV = nullptr, *dP = nullptr, *dW = nullptr, *dC = nullptr, *dN = nullptr;
  int32_t* dT = nullptr;
  // basis in box order and in canonical order
  int32_t *dPerm = nullptr, *dBtri = nullptr, *dBfv = nullptr;
  double *dBs = nullptr, *dBd = nullptr;
  int32_t *dCtri = nullptr, *dCfv = nullptr;
  double* dCs = nullptr;
  // near field
  // near field: RWG-RWG blocks (NJ) and triangle-triangle blocks of the
  // scalar operator (NT), each stored as its upper triangle
  pie::DevNear NJ{}, NT{};
  void *dNearJ = nullptr, *dNearT = nullptr;
  int64_t near_entries = 0, near_entries_J = 0, near_entries_T = 0;
  int64_t near_stored_J = 0, near_stored_T = 0, nslots_J = 0, nslots_T = 0;
  int32_t *dPermJ = nullptr, *dPermT = nullptr;  // RWG / triangle slots -> canonical RWG / triangle
  int32_t* dBoxPtr = nullptr;                    // [nbL+1] box-order unknown ranges
  pie::DevTriDiv TD{};                           // divergence sources of the triangles
  // second stream for the near field, forked from and joined to the caller's
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // third stream: the finest level's interaction-list translation, which
  // needs only the finest patterns and overlaps the upward shifts
  hipStream_t side2 = nullptr;
  hipEvent_t ev_agg = nullptr, ev_il = nullptr;
  // one stream per level 4..L for translations forked as soon as the
  // level's patterns exist (il_fork 3), with their fork and join events
  std::vector<hipStream_t> il_st;
  std::vector<hipEvent_t> ev_s, ev_g;
  // launch schedule (every choice gives the same result, bit for bit)
  int sched_near = PIE_NEAR_FORK_START;  // where the near field forks off the far chain
  int sched_il = 1;                      // finest translation on the third stream
  int sched_chunk = 4;                   // widest RHS chunk (1, 2 or 4; at most rc)
  bool force_ms = false;                 // PIE_OPT_MATRIX_SHIFTS
  // incidences
  pie::DevInc I{};
  int64_t ninc = 0;
  // levels (index l)
  std::vector<pie::DevLevel> lv;
  std::vector<double> s_l, kappa_l, d_l;
  std::vector<int> tau_l;  // truncation of Eq. (5) per level (>= 3)
  int64_t il_pairs = 0;
  // tables in far precision
  void* dM = nullptr;  // per-incidence moments [ninc][Qh][4] in far precision
  int Qh = 0;                   // samples stored in the moment table
  int32_t* dAnti = nullptr;     // [Q] stored sample of each sample (its antipode for q >= Qh)
  std::vector<void*> dTl, dFl, dFtl, dPhl;
  // workspace
  std::vector<void*> dS, dG;
  void *dPartJ = nullptr, *dPartT = nullptr;  // near partial sums [slot][W], [slot][2W]
  void *dXbJ = nullptr, *dXbT = nullptr;      // near inputs [E][W], [T][2W] (x_A, u)
  void* dPhi = nullptr;                       // per-triangle potentials [T][W] (FP64)
  double* dDiagScale = nullptr;  // |Z_uu|^-1/2, canonical order
  // block-diagonal preconditioner (inverses of the finest boxes' FP64 self
  // blocks, box order), built on the first solve that asks for it
  void* dPrec = nullptr;
  int64_t* dPrecOff = nullptr;
  double *dKhR = nullptr, *dPolR = nullptr, *dAmpR = nullptr, *dDirs = nullptr;
  int64_t ndirs_cap = 0;
  std::vector<void*> allocs;
  size_t bytes = 0;
  // stage profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
  ~pie_op() {
    if (side) (void)hipStreamDestroy(side);
    if (side2) (void)hipStreamDestroy(side2);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_agg) (void)hipEventDestroy(ev_agg);
    if (ev_il) (void)hipEventDestroy(ev_il);
    for (hipStream_t x : il_st)
      if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t x : ev_s)
      if (x) (void)hipEventDestroy(x);
    for (hipEvent_t x : ev_g)
      if (x) (void)hipEventDestroy(x);
    for (auto& u : ev_used) {
      (void)hipEventDestroy(u.second.first);
      (void)hipEventDestroy(u.second.second);
    }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
  }
};

// Widest MVM pass: the far-field workspace holds this many RHS columns;
// wider batches run in several passes.
constexpr int kPassMax = 64;
// Passes of at least this many columns run the batched (matrix-core and
// grouped row translation) kernels.
constexpr int kBatchCols = 16;

struct pie_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~pie_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// Uneven batch: one stream and one completion event per object (default
// priority, non-blocking), forked from and joined back to the caller's
// stream on every call.
struct pie_batch {
  std::vector<pie_op*> ops;
  std::vector<hipStream_t> st;
  std::vector<hipEvent_t> done;
  hipEvent_t start = nullptr;
  ~pie_batch() {
    for (hipStream_t s : st) (void)hipStreamDestroy(s);
    for (hipEvent_t e : done) (void)hipEventDestroy(e);
    if (start) (void)hipEventDestroy(start);
  }
};

namespace {

using namespace pie;

pie_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? PIE_ERR_OOM : PIE_ERR_HIP;
}

#define HIPCHK(expr, what)                    \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

template <typename T>
pie_status dalloc(pie_op* op, T** p, size_t n) {
  void* q = nullptr;
  size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(e, "hipMalloc");
  }
  op->allocs.push_back(q);
  op->bytes += bytes;
  *p = (T*)q;
  return PIE_OK;
}

template <typename T>
pie_status upload(pie_op* op, T** p, const std::vector<T>& h) {
  pie_status s = dalloc(op, p, h.size());
  if (s) return s;
  if (!h.empty()) HIPCHK(hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
  return PIE_OK;
}

template <typename T>
std::vector<T> narrow32(const std::vector<int64_t>& v) {
  return std::vector<T>(v.begin(), v.end());
}

// 7-point degree-5 triangle rule (Radon): barycentric nodes and weights.
void radon7(double bary[7][3], double w[7]) {
  const double s15 = std::sqrt(15.0);
  const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
  const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
  const double b[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, a1, 1 - 2 * a1}, {a1, 1 - 2 * a1, a1},
                          {1 - 2 * a1, a1, a1},         {a2, a2, 1 - 2 * a2}, {a2, 1 - 2 * a2, a2},
                          {1 - 2 * a2, a2, a2}};
  const double ww[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
  for (int i = 0; i < 7; ++i) {
    for (int k = 0; k < 3; ++k) bary[i][k] = b[i][k];
    w[i] = ww[i];
  }
}

double dfact(int n) {  // n!! for odd n >= -1
  double r = 1.0;
  for (int i = n; i > 1; i -= 2) r *= i;
  return r;
}

template <typename TF>
std::vector<TF> cast_vec(const std::vector<double>& v) {
  return std::vector<TF>(v.begin(), v.end());
}

template <typename TF>
pie_status upload_tables(pie_op* op, const std::vector<double>& khat, const std::vector<std::vector<double>>& T,
                         const std::vector<std::vector<double>>& F, const std::vector<std::vector<double>>& Ph) {
  pie_status s = PIE_OK;
  (void)khat;
  op->dTl.assign(op->L + 1, nullptr);
  op->dFl.assign(op->L + 1, nullptr);
  op->dFtl.assign(op->L + 1, nullptr);
  op->dPhl.assign(op->L + 1, nullptr);
  static_assert(TRANSLATE_OFFSETS == kNumOffsets, "offset table size");
  for (int l = 3; l <= op->L; ++l) {
    TF* t = nullptr;
    if ((s = upload(op, &t, cast_vec<TF>(T[l])))) return s;
    op->dTl[l] = t;
    if (l < op->L) {
      // both layouts padded with SQT zeros (row tiles of the shift kernels)
      const int Q = op->Q;
      std::vector<double> Fp(F[l]);
      Fp.resize((size_t)Q * Q + SQT, 0.0);
      TF* f = nullptr;
      if ((s = upload(op, &f, cast_vec<TF>(Fp)))) return s;
      op->dFl[l] = f;
      std::vector<double> Ftr((size_t)Q * Q + SQT, 0.0);
      for (int a = 0; a < Q; ++a)
        for (int b = 0; b < Q; ++b) Ftr[(size_t)b * Q + a] = F[l][(size_t)a * Q + b];
      TF* ft = nullptr;
      if ((s = upload(op, &ft, cast_vec<TF>(Ftr)))) return s;
      op->dFtl[l] = ft;
      TF* ph = nullptr;
      if ((s = upload(op, &ph, cast_vec<TF>(Ph[l])))) return s;
      op->dPhl[l] = ph;
    }
  }
  return PIE_OK;
}

// One near-field structure (kind 0: RWG-RWG, 1: triangle-triangle) over
// per-box slot counts cnt.  A finest box's slots are cut into near boxes of
// at most kNearBox slots (runs of its box order), so that every stored block
// fits the SpMM's 128-row / 128-column tiles whatever a finest box holds;
// near box v covers slots [sptr[v], sptr[v] + n_v) starting at box-order
// unknown ubase_v, and vptr[b] .. vptr[b + 1] are the near boxes of finest
// box b.  Stored blocks (v <= w, the finest boxes near) are grouped by row
// near box and split into row panels of at most one LDS panel (2048 FP32 /
// 1024 FP64 entries), one SpMM work unit each; row_ptr / col_ptr receive the
// per-near-box join ranges and vptr the near boxes of each finest box (host
// copies).
constexpr int kNearBox = 128;
// Most RWG functions or triangles in one finest box.
constexpr int kMaxBoxSlots = 32 * kNearBox;
pie_status build_near(pie_op* op, const Tree& t, int kind, const std::vector<int32_t>& cnt_box,
                      const std::vector<int32_t>& ubase_box, DevNear& out, int64_t& stored, int64_t& entries,
                      int64_t& nslots, std::vector<int32_t>& row_ptr, std::vector<int32_t>& col_ptr,
                      std::vector<int32_t>& vptr) {
  const int nbox = (int)cnt_box.size();
  std::vector<int32_t> cnt, ubase, vreal;
  vptr.assign(nbox + 1, 0);
  for (int b = 0; b < nbox; ++b) {
    for (int c = 0; c * kNearBox < cnt_box[b]; ++c) {
      cnt.push_back(std::min(kNearBox, cnt_box[b] - c * kNearBox));
      ubase.push_back(ubase_box[b] + c * kNearBox);
      vreal.push_back(b);
    }
    vptr[b + 1] = (int32_t)cnt.size();
  }
  const int nbL = (int)cnt.size();
  std::vector<int32_t> sptr(nbL + 1, 0);
  for (int b = 0; b < nbL; ++b) sptr[b + 1] = sptr[b] + cnt[b];
  const int zcap = op->near_prec == PIE_FP32 ? 2048 : 1024;
  std::vector<int32_t> ba, bb, prow, col_blk, tpc;
  row_ptr.assign(nbL + 1, 0);
  col_ptr.assign(nbL + 1, 0);
  std::vector<NearTaskDesc> tdesc;
  std::vector<int64_t> boff;
  std::vector<std::vector<int32_t>> cols(nbL);
  int64_t off = 0, slot = 0, ent = 0;
  for (int a = 0; a < nbL; ++a) {
    const int A = vreal[a];
    for (int64_t k = t.near_ptr[A]; k < t.near_ptr[A + 1]; ++k)
    for (int b = vptr[t.near_idx[k]]; b < vptr[t.near_idx[k] + 1]; ++b) {
      const int na = cnt[a], nb = cnt[b];
      if (b < a || na == 0 || nb == 0) continue;
      const int id = (int)ba.size();
      ba.push_back(a);
      bb.push_back(b);
      boff.push_back(off);
      // rows stored with an odd stride nb | 1, so that the SpMM's row-wise
      // LDS reads (one row per lane) hit distinct banks
      const int ldz = nb | 1;
      off += ((int64_t)na * ldz + 3) & ~int64_t(3);  // 4-entry (32-byte FP32) aligned blocks
      ent += (int64_t)na * nb;
      prow.push_back((int32_t)slot);
      slot += na;
      // one panel when the block fits, else the fewest equal panels (even
      // row counts for FP32, so that panel starts stay 16-byte aligned)
      const int cap = std::max(1, std::min(128, zcap / ldz));
      int rpp = na;
      if (na > cap) {
        for (int npn = (na + cap - 1) / cap;; ++npn) {
          rpp = (na + npn - 1) / npn;
          if (op->near_prec == PIE_FP32 && (rpp & 1)) ++rpp;
          if (rpp <= cap) break;
        }
      }
      for (int i0 = 0; i0 < na; i0 += rpp) {
        const int tid_ = (int)tdesc.size();
        NearTaskDesc d;
        d.off = boff[id] + (int64_t)i0 * ldz;
        d.v0 = sptr[b];
        d.nb = nb;
        d.ua = sptr[a] + i0;
        d.nr = std::min(na, i0 + rpp) - i0;
        d.prow = prow[id] + i0;
        if (b != a) {
          d.pcol = (int32_t)slot;
          slot += nb;
          cols[b].push_back(tid_);
        } else {
          d.pcol = -1;
        }
        tpc.push_back(d.pcol);
        tdesc.push_back(d);
      }
    }
    row_ptr[a + 1] = (int32_t)ba.size();
  }
  for (int b = 0; b < nbL; ++b) {
    col_ptr[b + 1] = col_ptr[b] + (int32_t)cols[b].size();
    col_blk.insert(col_blk.end(), cols[b].begin(), cols[b].end());
  }
  stored = off;
  entries = ent;
  nslots = slot;
  int32_t *dba, *dbb, *dprow, *dsp, *dub, *drp, *dcp, *dcb, *dtpc;
  int64_t* dbo;
  NearTaskDesc* dtd;
  pie_status s;
  int32_t* dvp;
  if ((s = upload(op, &dba, ba)) || (s = upload(op, &dbb, bb)) || (s = upload(op, &dbo, boff)) ||
      (s = upload(op, &dprow, prow)) || (s = upload(op, &dsp, sptr)) || (s = upload(op, &dub, ubase)) ||
      (s = upload(op, &drp, row_ptr)) || (s = upload(op, &dcp, col_ptr)) || (s = upload(op, &dcb, col_blk)) ||
      (s = upload(op, &dtd, tdesc)) || (s = upload(op, &dtpc, tpc)) || (s = upload(op, &dvp, vptr)))
    return s;
  out = DevNear{kind, (int32_t)ba.size(), dba, dbb, dbo, dprow, (int32_t)tdesc.size(), dtd, dtpc,
                dsp, dub, dvp, drp, dcp, dcb};
  return PIE_OK;
}

pie_status build_operator(pie_op* op, hipStream_t st) {
  const Mesh& m = *op->mesh;
  const Tree& t = *op->tree;
  pie_status s;
  const int N = op->N, ne = op->ne, nt = op->nt, L = op->L;
  // ---------------- geometry
  double bary[7][3], rw[7];
  radon7(bary, rw);
  std::vector<double> P(21 * (size_t)nt), W(7 * (size_t)nt);
  for (int tt = 0; tt < nt; ++tt) {
    const double* v0 = &m.V[3 * m.T[3 * tt]];
    const double* v1 = &m.V[3 * m.T[3 * tt + 1]];
    const double* v2 = &m.V[3 * m.T[3 * tt + 2]];
    for (int i = 0; i < 7; ++i) {
      for (int d = 0; d < 3; ++d) P[21 * tt + 3 * i + d] = bary[i][0] * v0[d] + bary[i][1] * v1[d] + bary[i][2] * v2[d];
      W[7 * tt + i] = m.area[tt] * rw[i];
    }
  }
  if ((s = upload(op, &op->dV, m.V))) return s;
  if ((s = upload(op, &op->dT, m.T))) return s;
  if ((s = upload(op, &op->dP, P))) return s;
  if ((s = upload(op, &op->dW, W))) return s;
  if ((s = upload(op, &op->dC, m.centroid))) return s;
  if ((s = upload(op, &op->dN, m.normal))) return s;
  DevGeo G{op->dV, op->dT, op->dP, op->dW, op->dC, op->dN, (int32_t)nt};
  // ---------------- basis (box order and canonical)
  std::vector<int32_t> perm(N), btri(2 * (size_t)N), bfv(2 * (size_t)N, -1);
  std::vector<double> bs(2 * (size_t)N, 0.0), bd(2 * (size_t)N, 0.0);
  std::vector<int32_t> ctri(2 * (size_t)ne), cfv(2 * (size_t)ne);
  std::vector<double> cs(2 * (size_t)ne);
  for (int e = 0; e < ne; ++e)
    for (int h = 0; h < 2; ++h) {
      int tr = m.etri[2 * e + h];
      double sg = h == 0 ? 1.0 : -1.0;
      ctri[2 * e + h] = tr;
      cfv[2 * e + h] = m.efree[2 * e + h];
      cs[2 * e + h] = sg * m.elen[e] / (2.0 * m.area[tr]);
    }
  for (int u = 0; u < N; ++u) {
    int cu = (int)t.perm[u];
    perm[u] = cu;
    if (cu < ne) {
      for (int h = 0; h < 2; ++h) {
        int tr = m.etri[2 * cu + h];
        double sg = h == 0 ? 1.0 : -1.0;
        btri[2 * u + h] = tr;
        bfv[2 * u + h] = m.efree[2 * cu + h];
        bs[2 * u + h] = sg * m.elen[cu] / (2.0 * m.area[tr]);
        bd[2 * u + h] = sg * m.elen[cu] / m.area[tr];
      }
    } else {
      btri[2 * u] = btri[2 * u + 1] = cu - ne;
    }
  }
  if ((s = upload(op, &op->dPerm, perm))) return s;
  if ((s = upload(op, &op->dBtri, btri))) return s;
  if ((s = upload(op, &op->dBfv, bfv))) return s;
  if ((s = upload(op, &op->dBs, bs))) return s;
  if ((s = upload(op, &op->dBd, bd))) return s;
  if ((s = upload(op, &op->dCtri, ctri))) return s;
  if ((s = upload(op, &op->dCfv, cfv))) return s;
  if ((s = upload(op, &op->dCs, cs))) return s;
  DevBasis B{op->dPerm, op->dBtri, op->dBfv, op->dBs, op->dBd, N, ne};
  // ---------------- near blocks (upper triangle, grouped by row box): the
  // RWG-RWG blocks over the boxes' RWG slots and the triangle-triangle blocks
  // of the scalar operator over their triangle slots (each box's RWG
  // functions come first in box order, then its triangles)
  const Level& fl = t.lev[L];
  const int nbL = (int)fl.nb;
  std::vector<int32_t> box_ptr = narrow32<int32_t>(t.box_ptr);
  std::vector<int32_t> cntJ(nbL, 0), cntT(nbL, 0), permJ, permT;
  for (int b = 0; b < nbL; ++b)
    for (int u = box_ptr[b]; u < box_ptr[b + 1]; ++u) {
      if (perm[u] < ne) {
        ++cntJ[b];
        permJ.push_back(perm[u]);
      } else {
        ++cntT[b];
        permT.push_back(perm[u] - ne);
      }
    }
  for (int b = 0; b < nbL; ++b)
    if (cntJ[b] > kMaxBoxSlots || cntT[b] > kMaxBoxSlots) {
      set_error("a finest box holds more than " + std::to_string(kMaxBoxSlots) +
                " RWG functions or triangles; use more levels");
      return PIE_ERR_UNSUPPORTED;
    }
  if ((s = upload(op, &op->dPermJ, permJ)) || (s = upload(op, &op->dPermT, permT)) ||
      (s = upload(op, &op->dBoxPtr, box_ptr)))
    return s;
  std::vector<int32_t> row_ptr_J, col_ptr_J, row_ptr_T, col_ptr_T, vptr_J, vptr_T;
  int64_t entJ = 0, entT = 0;
  {
    std::vector<int32_t> ubJ(nbL), ubT(nbL);
    for (int b = 0; b < nbL; ++b) {
      ubJ[b] = box_ptr[b];
      ubT[b] = box_ptr[b] + cntJ[b];
    }
    if ((s = build_near(op, t, 0, cntJ, ubJ, op->NJ, op->near_stored_J, entJ, op->nslots_J, row_ptr_J, col_ptr_J,
                        vptr_J)) ||
        (s = build_near(op, t, 1, cntT, ubT, op->NT, op->near_stored_T, entT, op->nslots_T, row_ptr_T, col_ptr_T,
                        vptr_T)))
      return s;
  }
  op->near_entries = entJ + entT;
  op->near_entries_J = entJ;
  op->near_entries_T = entT;
  // divergence sources of every triangle (canonical): the RWG functions on
  // its edges with +-l/A (the same value as the box-order divergences)
  {
    std::vector<int32_t> te(3 * (size_t)nt, -1);
    std::vector<double> td(3 * (size_t)nt, 0.0);
    std::vector<int> fill(nt, 0);
    for (int e = 0; e < ne; ++e)
      for (int h = 0; h < 2; ++h) {
        const int tr = m.etri[2 * e + h];
        const int k = fill[tr]++;
        te[3 * (size_t)tr + k] = e;
        td[3 * (size_t)tr + k] = (h == 0 ? 1.0 : -1.0) * m.elen[e] / m.area[tr];
      }
    int32_t* dte;
    double* dtd;
    if ((s = upload(op, &dte, te)) || (s = upload(op, &dtd, td))) return s;
    op->TD = DevTriDiv{dte, dtd, (int32_t)nt, (int32_t)ne};
  }
  // ---------------- incidences
  std::vector<int32_t> iptr(nbL + 1, 0), itri, irwg, ifv, ipulse, uslot(2 * (size_t)N, -1);
  std::vector<double> irs;
  int maxinc = 0;
  for (int b = 0; b < nbL; ++b) {
    std::map<int, int> local;  // triangle -> incidence index
    auto get = [&](int tr) {
      auto it = local.find(tr);
      if (it != local.end()) return it->second;
      int j = (int)itri.size();
      itri.push_back(tr);
      for (int k = 0; k < 3; ++k) {
        irwg.push_back(-1);
        ifv.push_back(0);
        irs.push_back(0.0);
      }
      ipulse.push_back(-1);
      local[tr] = j;
      return j;
    };
    for (int u = box_ptr[b]; u < box_ptr[b + 1]; ++u) {
      if (perm[u] < ne) {
        for (int h = 0; h < 2; ++h) {
          int j = get(btri[2 * u + h]);
          int k = 0;
          while (irwg[3 * j + k] >= 0) ++k;  // at most three edges per triangle
          irwg[3 * j + k] = u;
          irs[3 * j + k] = bs[2 * u + h];
          ifv[3 * j + k] = bfv[2 * u + h];
          uslot[2 * u + h] = 4 * j + k;
        }
      } else {
        int j = get(btri[2 * u]);
        ipulse[j] = u;
        uslot[2 * u] = uslot[2 * u + 1] = 4 * j + 3;
      }
    }
    iptr[b + 1] = (int32_t)itri.size();
    maxinc = std::max(maxinc, iptr[b + 1] - iptr[b]);
  }
  op->ninc = (int64_t)itri.size();
  op->maxinc = maxinc;
  {
    // geometry relative to the finest box centre (the same centre formula
    // as the level tables below)
    const Level& LL = t.lev[L];
    const double dL = t.side / (double)(int64_t(1) << (L - 1));
    auto centre = [&](int b, int c) { return t.origin[c] + ((double)LL.coords[3 * b + c] + 0.5) * dL; };
    const size_t ni = itri.size();
    std::vector<double> ipw(28 * ni), ipv(9 * ni, 0.0);
    std::vector<int32_t> ixc(4 * ni, -1);
    std::vector<int32_t> uj(2 * (size_t)N, 0);
    std::vector<double> us(2 * (size_t)N, 0.0), upv(6 * (size_t)N, 0.0);
    for (int b = 0; b < nbL; ++b) {
      const double C[3] = {centre(b, 0), centre(b, 1), centre(b, 2)};
      for (int j = iptr[b]; j < iptr[b + 1]; ++j) {
        const int tr = itri[j];
        for (int i = 0; i < 7; ++i) {
          for (int c = 0; c < 3; ++c) ipw[28 * (size_t)j + 4 * i + c] = P[21 * (size_t)tr + 3 * i + c] - C[c];
          ipw[28 * (size_t)j + 4 * i + 3] = W[7 * (size_t)tr + i];
        }
        for (int k = 0; k < 3; ++k) {
          const int u = irwg[3 * j + k];
          if (u < 0) {
            irs[3 * j + k] = 0.0;
            continue;
          }
          ixc[4 * (size_t)j + k] = perm[u];
          for (int c = 0; c < 3; ++c) ipv[9 * (size_t)j + 3 * k + c] = m.V[3 * (size_t)ifv[3 * j + k] + c] - C[c];
        }
        if (ipulse[j] >= 0) ixc[4 * (size_t)j + 3] = perm[ipulse[j]];
      }
      for (int u = box_ptr[b]; u < box_ptr[b + 1]; ++u)
        for (int h = 0; h < 2; ++h) {
          const int slot = uslot[2 * u + h];
          const int j = slot >> 2, k = slot & 3;
          uj[2 * u + h] = j;
          if (k == 3) continue;
          us[2 * u + h] = irs[3 * j + k];
          for (int c = 0; c < 3; ++c) upv[6 * (size_t)u + 3 * h + c] = m.V[3 * (size_t)ifv[3 * j + k] + c] - C[c];
        }
    }
    int32_t *dip, *dxc, *duj;
    double *dpw, *drs, *dpv, *dus, *dupv;
    if ((s = upload(op, &dip, iptr)) || (s = upload(op, &dpw, ipw)) || (s = upload(op, &dxc, ixc)) ||
        (s = upload(op, &drs, irs)) || (s = upload(op, &dpv, ipv)) || (s = upload(op, &duj, uj)) ||
        (s = upload(op, &dus, us)) || (s = upload(op, &dupv, upv)))
      return s;
    op->I = DevInc{dip, dpw, dxc, drs, dpv, duj, dus, dupv, op->dBoxPtr, op->TD};
  }
  // longest near-field join list of a finest box (partial-sum slots of its
  // near boxes and their ranges, staged in LDS by the reception)
  op->maxjoin = 0;
  for (int b = 0; b < nbL; ++b) {
    int n = (vptr_J[b + 1] - vptr_J[b]) + (vptr_T[b + 1] - vptr_T[b]) + 2;
    for (int v = vptr_J[b]; v < vptr_J[b + 1]; ++v)
      n += (row_ptr_J[v + 1] - row_ptr_J[v]) + (col_ptr_J[v + 1] - col_ptr_J[v]);
    for (int v = vptr_T[b]; v < vptr_T[b + 1]; ++v)
      n += (row_ptr_T[v + 1] - row_ptr_T[v]) + (col_ptr_T[v + 1] - col_ptr_T[v]);
    op->maxjoin = std::max(op->maxjoin, n);
  }
  // ---------------- levels
  op->lv.assign(L + 1, DevLevel{});
  op->s_l.assign(L + 1, 0.0);
  op->kappa_l.assign(L + 1, 0.0);
  op->d_l.assign(L + 1, 0.0);
  op->il_pairs = 0;
  for (int l = 3; l <= L; ++l) {
    const Level& lvh = t.lev[l];
    const int nb = (int)lvh.nb;
    for (int b = 0; b < nb; ++b)
      if (lvh.il_ptr[b + 1] - lvh.il_ptr[b] > IL_MAX) {
        set_error("interaction list longer than the one-box-buffer bound");
        return PIE_ERR_MESH;
      }
    const double d = t.side / (double)(int64_t(1) << (l - 1));
    op->d_l[l] = d;
    op->s_l[l] = std::min(1.0, op->k * d / op->xs);
    op->kappa_l[l] = op->k / op->s_l[l];
    std::vector<double> cen(3 * (size_t)nb);
    std::vector<int32_t> oct(nb);
    for (int b = 0; b < nb; ++b) {
      for (int c = 0; c < 3; ++c) cen[3 * b + c] = t.origin[c] + ((double)lvh.coords[3 * b + c] + 0.5) * d;
      oct[b] = (int32_t)((lvh.coords[3 * b] & 1) | ((lvh.coords[3 * b + 1] & 1) << 1) |
                         ((lvh.coords[3 * b + 2] & 1) << 2));
    }
    DevLevel dl{};
    dl.nb = nb;
    double* dcen;
    int32_t *dpar, *doct, *dchild = nullptr, *dilp, *dils, *dilo;
    if ((s = upload(op, &dcen, cen)) || (s = upload(op, &dpar, narrow32<int32_t>(lvh.parent))) ||
        (s = upload(op, &doct, oct)) || (s = upload(op, &dilp, narrow32<int32_t>(lvh.il_ptr))) ||
        (s = upload(op, &dils, narrow32<int32_t>(lvh.il_src))) ||
        (s = upload(op, &dilo, narrow32<int32_t>(lvh.il_off))))
      return s;
    if (l < L && (s = upload(op, &dchild, narrow32<int32_t>(lvh.child_ptr)))) return s;
    // parent groups of the upward shift: runs of parents with at most
    // SHIFT_GROUP children in total
    int32_t* dug = nullptr;
    int32_t nug = 0;
    if (l < L) {
      std::vector<int32_t> ug{0};
      int64_t cnt = 0;
      for (int p = 0; p < nb; ++p) {
        const int64_t nc = lvh.child_ptr[p + 1] - lvh.child_ptr[p];
        if (cnt + nc > SHIFT_GROUP) {
          ug.push_back(p);
          cnt = 0;
        }
        cnt += nc;
      }
      ug.push_back(nb);
      nug = (int32_t)ug.size() - 1;
      if ((s = upload(op, &dug, ug))) return s;
    }
    dl.centre = dcen;
    dl.parent = dpar;
    dl.octant = doct;
    dl.child_ptr = dchild;
    dl.il_ptr = dilp;
    dl.il_src = dils;
    dl.il_off = dilo;
    dl.nug = nug;
    dl.ug_ptr = dug;
    {
      // translation groups: runs of boxes with one parent (children are
      // contiguous in Morton order) cut into near-equal parts of at most
      // TG_BOXES boxes; per group the ascending union of its sources, each
      // with the offset index of every box that lists it
      std::vector<int32_t> tg{0}, tgent{0};
      std::vector<int4> te;
      auto add_group = [&](int b0, int b1) {
        std::vector<std::pair<int32_t, int32_t>> ent;  // (source, box slot << 16 | offset)
        for (int b = b0; b < b1; ++b)
          for (int64_t e = lvh.il_ptr[b]; e < lvh.il_ptr[b + 1]; ++e)
            ent.push_back({(int32_t)lvh.il_src[e], ((b - b0) << 16) | (int32_t)lvh.il_off[e]});
        std::sort(ent.begin(), ent.end());
        for (size_t i = 0; i < ent.size();) {
          uint32_t o[TG_BOXES];
          for (int d = 0; d < TG_BOXES; ++d) o[d] = 0xffffu;
          const int32_t u = ent[i].first;
          for (; i < ent.size() && ent[i].first == u; ++i) o[ent[i].second >> 16] = ent[i].second & 0xffff;
          te.push_back(make_int4(u, (int32_t)(o[0] | (o[1] << 16)), (int32_t)(o[2] | (o[3] << 16)), 0));
        }
        tg.push_back(b1);
        tgent.push_back((int32_t)te.size());
      };
      for (int b0 = 0; b0 < nb;) {
        int b1 = b0 + 1;
        while (b1 < nb && lvh.parent[b1] == lvh.parent[b0]) ++b1;
        const int n = b1 - b0, parts = (n + TG_BOXES - 1) / TG_BOXES;
        for (int p = 0, s0 = b0; p < parts; ++p) {
          const int s1 = s0 + (n - (s0 - b0) + (parts - p) - 1) / (parts - p);
          add_group(s0, s1);
          s0 = s1;
        }
        b0 = b1;
      }
      int32_t *dtg, *dtge;
      int4* dte;
      if ((s = upload(op, &dtg, tg)) || (s = upload(op, &dtge, tgent)) || (s = upload(op, &dte, te))) return s;
      dl.ntg = (int32_t)tg.size() - 1;
      dl.tg_box = dtg;
      dl.tg_ent = dtge;
      dl.te = dte;
    }
    op->lv[l] = dl;
    op->il_pairs += (int64_t)lvh.il_src.size();
  }
  // ---------------- k-space samples and tables (FP64)
  const int Q = op->Q;
  std::vector<double> ct, wt;
  gauss_legendre(op->nth, ct, wt);
  std::vector<double> khat(3 * (size_t)Q), wq(Q);
  for (int i = 0; i < op->nth; ++i)
    for (int j = 0; j < op->nph; ++j) {
      int q = i * op->nph + j;
      double ph = 2.0 * kPi * j / op->nph;
      double st_ = std::sqrt(1.0 - ct[i] * ct[i]);
      khat[3 * q] = st_ * std::cos(ph);
      khat[3 * q + 1] = st_ * std::sin(ph);
      khat[3 * q + 2] = ct[i];
      wq[q] = wt[i] * (2.0 * kPi / op->nph);
    }
  // translation tables T_l[off][q] = (ik/16pi^2) w_q alpha~(khat_q, w = off d_l)
  std::vector<std::vector<double>> Tt(L + 1), Ft(L + 1), Pht(L + 1);
  double tmax = 0.0;
  for (int l = 3; l <= L; ++l) {
    Tt[l].assign(2 * (size_t)kNumOffsets * Q, 0.0);
    int id = 0;
    for (int a = -3; a <= 3; ++a)
      for (int b = -3; b <= 3; ++b)
        for (int c = -3; c <= 3; ++c) {
          if (std::max({std::abs(a), std::abs(b), std::abs(c)}) < 2) continue;
          double wv[3] = {a * op->d_l[l], b * op->d_l[l], c * op->d_l[l]};
          double wn = std::sqrt(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
          std::vector<double> hk;
          scaled_hankel(op->k, op->s_l[l], wn, op->tau_l[l], hk);  // k s^t h_t
          for (int q = 0; q < Q; ++q) {
            double x = (khat[3 * q] * wv[0] + khat[3 * q + 1] * wv[1] + khat[3 * q + 2] * wv[2]) / wn;
            std::complex<double> acc(0.0, 0.0);
            double p0 = 1.0, p1 = x;
            std::complex<double> it(1.0, 0.0);  // i^t
            for (int tt = 0; tt <= op->tau_l[l]; ++tt) {
              double Pt = tt == 0 ? 1.0 : (tt == 1 ? x : 0.0);
              if (tt >= 2) {
                double p2 = ((2.0 * tt - 1.0) * x * p1 - (tt - 1.0) * p0) / tt;
                p0 = p1;
                p1 = p2;
                Pt = p2;
              }
              acc += it * (2.0 * tt + 1.0) * std::complex<double>(hk[2 * tt], hk[2 * tt + 1]) * Pt;
              it *= std::complex<double>(0.0, 1.0);
            }
            std::complex<double> v = std::complex<double>(0.0, 1.0) / (16.0 * kPi * kPi) * wq[q] * acc;
            Tt[l][2 * ((size_t)id * Q + q)] = v.real();
            Tt[l][2 * ((size_t)id * Q + q) + 1] = v.imag();
            tmax = std::max(tmax, std::abs(v));
          }
          ++id;
        }
    if (l < L) {
      // inter-level filter F[q][q'] = w_q' sum_l (2l+1)/4pi ratio^l P_l(khat_q.khat_q'),
      // degrees up to the parent level's truncation
      const double ratio = op->kappa_l[l] / op->kappa_l[l + 1];
      Ft[l].assign((size_t)Q * Q, 0.0);
      for (int q = 0; q < Q; ++q)
        for (int qq = 0; qq < Q; ++qq) {
          double x = khat[3 * q] * khat[3 * qq] + khat[3 * q + 1] * khat[3 * qq + 1] + khat[3 * q + 2] * khat[3 * qq + 2];
          x = std::max(-1.0, std::min(1.0, x));
          double p0 = 1.0, p1 = x, sum = 1.0 / (4.0 * kPi), rp = 1.0;
          for (int ll = 1; ll <= op->tau_l[l]; ++ll) {
            double Pl;
            if (ll == 1) {
              Pl = x;
            } else {
              Pl = ((2.0 * ll - 1.0) * x * p1 - (ll - 1.0) * p0) / ll;
              p0 = p1;
              p1 = Pl;
            }
            rp *= ratio;
            sum += (2.0 * ll + 1.0) / (4.0 * kPi) * rp * Pl;
          }
          Ft[l][(size_t)q * Q + qq] = sum * wq[qq];
        }
      // child phases exp(-i kappa_l khat_q . (C_child - C_parent)), per octant
      Pht[l].assign(2 * 8 * (size_t)Q, 0.0);
      const double dc = op->d_l[l] / 2.0;
      for (int o = 0; o < 8; ++o) {
        double del[3] = {((o & 1) - 0.5) * dc, (((o >> 1) & 1) - 0.5) * dc, (((o >> 2) & 1) - 0.5) * dc};
        for (int q = 0; q < Q; ++q) {
          double th = op->kappa_l[l] * (khat[3 * q] * del[0] + khat[3 * q + 1] * del[1] + khat[3 * q + 2] * del[2]);
          Pht[l][2 * ((size_t)o * Q + q)] = std::cos(th);
          Pht[l][2 * ((size_t)o * Q + q) + 1] = -std::sin(th);
        }
      }
    }
  }
  if (op->far_prec == PIE_FP32 && !(tmax < 1e30)) {
    set_error("translation table exceeds the FP32 range");
    return PIE_ERR_PRECISION;
  }
  s = op->far_prec == PIE_FP32 ? upload_tables<float>(op, khat, Tt, Ft, Pht)
                               : upload_tables<double>(op, khat, Tt, Ft, Pht);
  if (s) return s;
  // ---------------- chunk width for the RHS loop: LDS budget 64 KiB (four
  // workgroups per CU); boxes with more incidences (coarse trees) take one
  // column at a time with up to the device's per-workgroup LDS
  const int tfb = op->far_prec == PIE_FP32 ? 4 : 8;
  int lds_max = 65536;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, op->device) != hipSuccess ||
      lds_max < 65536)
    lds_max = 65536;
  op->lds_budget = 65536;
  op->rc = 0;
  for (int rc : {4, 2, 1}) {
    if (rc > op->max_rhs && rc > 1) continue;
    size_t a = aggregate_smem(op->maxinc, Q, 1, rc, tfb);
    size_t r = receive_smem(op->maxinc, Q, op->maxjoin, rc, tfb);
    if (a <= 65536 && r <= 65536) {
      op->rc = rc;
      break;
    }
  }
  if (op->rc == 0 && aggregate_smem(op->maxinc, Q, 1, 1, tfb) <= (size_t)lds_max &&
      receive_smem(op->maxinc, Q, op->maxjoin, 1, tfb) <= (size_t)lds_max) {
    op->rc = 1;
    op->lds_budget = lds_max;
  }
  if (op->rc == 0) {
    set_error("a finest box has too many incidences for the LDS budget; use more levels");
    return PIE_ERR_UNSUPPORTED;
  }
  if (Q > 256) {
    set_error("more than 256 k-space samples per level are not supported");
    return PIE_ERR_UNSUPPORTED;
  }
  // ---------------- workspace (one pass of pw RHS columns)
  op->pw = std::min(op->max_rhs, kPassMax);
  const size_t cxf = 2 * (size_t)tfb, cxn = op->near_prec == PIE_FP32 ? 8 : 16;
  op->dS.assign(L + 1, nullptr);
  op->dG.assign(L + 1, nullptr);
  for (int l = 3; l <= L; ++l) {
    unsigned char *a, *b;
    size_t n = (size_t)op->lv[l].nb * Q * 5 * op->pw * cxf;
    if ((s = dalloc(op, &a, n)) || (s = dalloc(op, &b, n))) return s;
    op->dS[l] = a;
    op->dG[l] = b;
  }
  unsigned char *partJ, *partT, *xbJ, *xbT, *phi;
  if ((s = dalloc(op, &partJ, (size_t)op->nslots_J * op->pw * cxn)) ||
      (s = dalloc(op, &partT, (size_t)op->nslots_T * 2 * op->pw * cxn)) ||
      (s = dalloc(op, &xbJ, (size_t)ne * op->pw * cxn)) || (s = dalloc(op, &xbT, (size_t)nt * 2 * op->pw * cxn)) ||
      (s = dalloc(op, &phi, (size_t)nt * op->pw * 16)))
    return s;
  op->dPartJ = partJ;
  op->dPartT = partT;
  op->dXbJ = xbJ;
  op->dXbT = xbT;
  op->dPhi = phi;
  if ((s = dalloc(op, &op->dKhR, 3 * (size_t)op->max_rhs)) || (s = dalloc(op, &op->dPolR, 3 * (size_t)op->max_rhs)) ||
      (s = dalloc(op, &op->dAmpR, 2 * (size_t)op->max_rhs)))
    return s;
  // ---------------- finest-level moments of every incidence (FP64 phases).
  // With an even number of phi samples the sample set is closed under
  // khat -> -khat: (i, j) -> (n_theta-1-i, j + n_phi/2), and the first Q/2
  // samples hold one of each antipodal pair, so only they are stored.
  {
    std::vector<int32_t> anti(Q);
    op->Qh = Q;
    for (int q = 0; q < Q; ++q) anti[q] = q;
    if (op->nph % 2 == 0) {
      bool ok = true;
      for (int q = Q / 2; q < Q; ++q) {
        const int i = q / op->nph, j = q - i * op->nph;
        const int a = (op->nth - 1 - i) * op->nph + (j + op->nph / 2) % op->nph;
        double d = 0.0;
        for (int c = 0; c < 3; ++c) d = std::max(d, std::fabs(khat[3 * (size_t)q + c] + khat[3 * (size_t)a + c]));
        ok = ok && a < Q / 2 && d < 1e-14;
        anti[q] = a;
      }
      if (ok) {
        op->Qh = Q / 2;
      } else {
        for (int q = 0; q < Q; ++q) anti[q] = q;
      }
    }
    // aggregation: one lane per stored sample, nsplit incidence groups
    const int rcm = op->rc <= 1 ? 1 : (op->rc <= 2 ? 2 : 4);
    op->nsplit = 256 / op->Qh < 1 ? 1 : 256 / op->Qh;
    while (op->nsplit > 1 && aggregate_smem(op->maxinc, Q, op->nsplit, rcm, tfb) > (size_t)op->lds_budget)
      --op->nsplit;
    unsigned char* mt;
    double* dkh;
    if ((s = dalloc(op, &mt, (size_t)op->ninc * op->Qh * 4 * cxf)) || (s = upload(op, &dkh, khat)) ||
        (s = upload(op, &op->dAnti, anti)))
      return s;
    op->dM = mt;
    hipError_t em = op->far_prec == PIE_FP32
                        ? launch_moments<float>(op->I.pw, (int)op->ninc, dkh, op->Qh, op->kappa_l[L], mt, st)
                        : launch_moments<double>(op->I.pw, (int)op->ninc, dkh, op->Qh, op->kappa_l[L], mt, st);
    if (em != hipSuccess) return hip_fail(em, "moments launch");
  }
  // ---------------- near-field fill and diagonal (FP64 arithmetic)
  hipError_t e;
  for (int kind = 0; kind < 2; ++kind) {
    const int64_t stored = kind == 0 ? op->near_stored_J : op->near_stored_T;
    const DevNear& NS = kind == 0 ? op->NJ : op->NT;
    unsigned char* nz;
    if ((s = dalloc(op, &nz, (size_t)stored * cxn))) return s;
    (kind == 0 ? op->dNearJ : op->dNearT) = nz;
    HIPCHK(hipMemset(nz, 0, (size_t)stored * cxn), "near clear");  // row padding and block tails
    e = op->near_prec == PIE_FP32 ? launch_near_fill<float>(G, B, NS, nz, op->k, op->w2e, st)
                                  : launch_near_fill<double>(G, B, NS, nz, op->k, op->w2e, st);
    if (e != hipSuccess) return hip_fail(e, "near fill launch");
  }
  double* diag_box;
  if ((s = dalloc(op, &diag_box, N)) || (s = dalloc(op, &op->dDiagScale, N))) return s;
  if ((e = launch_diag(G, B, diag_box, op->k, op->w2e, st)) != hipSuccess) return hip_fail(e, "diag launch");
  HIPCHK(hipStreamSynchronize(st), "operator setup");
  std::vector<double> db(N), dsc(N);
  HIPCHK(hipMemcpy(db.data(), diag_box, N * sizeof(double), hipMemcpyDeviceToHost), "diag copy");
  for (int u = 0; u < N; ++u) dsc[perm[u]] = db[u] > 0.0 ? 1.0 / std::sqrt(db[u]) : 1.0;
  HIPCHK(hipMemcpy(op->dDiagScale, dsc.data(), N * sizeof(double), hipMemcpyHostToDevice), "diag copy");
  return PIE_OK;
}

hipEvent_t take_event(pie_op* op) {
  if (!op->ev_pool.empty()) {
    hipEvent_t e = op->ev_pool.back();
    op->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs one stage's launches, bracketed by events when profiling is on.
template <typename F>
hipError_t stage(pie_op* op, int id, hipStream_t st, F&& launch) {
  if (!op->prof) return launch();
  hipEvent_t a = take_event(op), b = take_event(op);
  if (!a || !b) return launch();
  (void)hipEventRecord(a, st);
  hipError_t e = launch();
  (void)hipEventRecord(b, st);
  op->ev_used.push_back({id, {a, b}});
  return e;
}

DevGeo geo(const pie_op* op) { return DevGeo{op->dV, op->dT, op->dP, op->dW, op->dC, op->dN, (int32_t)op->nt}; }
DevBasis basis(const pie_op* op) { return DevBasis{op->dPerm, op->dBtri, op->dBfv, op->dBs, op->dBd, op->N, op->ne}; }

// One chunk of <= rc right-hand sides; x, y point at the chunk's first
// column of [N][ld] arrays.  flags: 1 near, 2 far, 4 adjoint.
template <typename TF, typename TN>
pie_status mvm_chunk(pie_op* op, const void* x, void* y, int ld, int R, int flags, hipStream_t st) {
  const int L = op->L, Q = op->Q;
  const int rcap = std::min(op->rc, op->sched_chunk);  // widest register group of columns
  const bool near = flags & 1, far = flags & 2, adj = flags & 4;
  hipError_t e;
  // The near field runs either before the far chain on the caller's stream
  // or on the operator's side stream, forked at the start or after the
  // aggregation and joined before the reception.
  const bool fork = near && far && op->sched_near != PIE_NEAR_SERIAL;
  hipStream_t sn = fork ? op->side : st;
  auto near_field = [&]() -> pie_status {
    if (fork) {
      HIPCHK(hipEventRecord(op->ev_fork, st), "fork");
      HIPCHK(hipStreamWaitEvent(sn, op->ev_fork, 0), "fork");
    }
    if ((e = stage(op, PIE_STAGE_PERMUTE, sn, [&] {
           return launch_near_in<TN>(x, ld, op->dPermJ, op->dPermT, op->TD, op->w2e, R, adj, op->dXbJ, op->dXbT, sn);
         })) != hipSuccess)
      return hip_fail(e, "near input");
    // the scalar operator's blocks act on both x_A and u (2R columns); both
    // structures take the matrix-core path for batched passes
    const bool mf = R >= kBatchCols;
    if ((e = stage(op, PIE_STAGE_NEAR, sn, [&] {
           hipError_t e1 = launch_near_spmm<TN>(op->NJ, op->dNearJ, op->dXbJ, R, op->dPartJ, R, rcap, mf, sn);
           if (e1 != hipSuccess) return e1;
           return launch_near_spmm<TN>(op->NT, op->dNearT, op->dXbT, 2 * R, op->dPartT, 2 * R, rcap, mf, sn);
         })) != hipSuccess)
      return hip_fail(e, "near spmm");
    if (fork) HIPCHK(hipEventRecord(op->ev_join, sn), "join");
    return PIE_OK;
  };
  const bool near_late = fork && op->sched_near == PIE_NEAR_FORK_AFTER_AGGREGATE;
  if (near && !near_late) {
    pie_status ps = near_field();
    if (ps) return ps;
  }
  const DevBasis B = basis(op);
  if (far) {
    if ((e = stage(op, PIE_STAGE_AGGREGATE, st, [&] {
           return launch_aggregate<TF>(op->I, op->lv[L].nb, op->maxinc, x, ld, R, rcap, op->dM, op->dAnti, Q,
                                       op->Qh, op->w2e, adj, op->nsplit, op->dS[L], st);
         })) != hipSuccess)
      return hip_fail(e, "aggregate");
    if (near_late) {
      pie_status ps = near_field();
      if (ps) return ps;
    }
    // finest-level translation on the third stream, concurrent with the
    // upward shifts and the coarser translations; forked after the
    // aggregation (il_fork 1) or after the first upward shift (il_fork 2),
    // so that it overlaps the small coarse-level kernels instead.  il_fork 3
    // forks every level >= 4 to its own stream as soon as its patterns
    // exist and joins it before the downward shift into that level.
    const bool perlev = L > 3 && op->sched_il == 3;
    const bool fork2 = L > 3 && (op->sched_il == 1 || op->sched_il == 2);
    // il_fork 4: every level's translation in one launch after the upward
    // pass (no stream fork)
    const bool oneset = op->sched_il == 4;
    auto translate = [&](int l, hipStream_t s) {
      return stage(op, PIE_STAGE_TRANSLATE, s, [&] {
        return launch_translate<TF>(op->lv[l], op->dS[l], op->dTl[l], op->dG[l], Q, R, s);
      });
    };
    auto fork_translate = [&]() -> pie_status {
      HIPCHK(hipEventRecord(op->ev_agg, st), "fork");
      HIPCHK(hipStreamWaitEvent(op->side2, op->ev_agg, 0), "fork");
      if ((e = translate(L, op->side2)) != hipSuccess) return hip_fail(e, "translate");
      HIPCHK(hipEventRecord(op->ev_il, op->side2), "join");
      return PIE_OK;
    };
    auto fork_level = [&](int l) -> pie_status {
      HIPCHK(hipEventRecord(op->ev_s[l], st), "fork");
      HIPCHK(hipStreamWaitEvent(op->il_st[l], op->ev_s[l], 0), "fork");
      if ((e = translate(l, op->il_st[l])) != hipSuccess) return hip_fail(e, "translate");
      HIPCHK(hipEventRecord(op->ev_g[l], op->il_st[l]), "join");
      return PIE_OK;
    };
    if (perlev) {
      pie_status ps = fork_level(L);
      if (ps) return ps;
    }
    if (fork2 && op->sched_il == 1) {
      pie_status ps = fork_translate();
      if (ps) return ps;
    }
    for (int l = L - 1; l >= 3; --l) {
      if ((e = stage(op, PIE_STAGE_SHIFT_UP, st, [&] {
             return launch_shift_up<TF>(op->lv[l], op->lv[l + 1], op->dS[l + 1], op->dS[l], op->dFtl[l],
                                        op->dPhl[l], Q, R, op->force_ms, st);
           })) != hipSuccess)
        return hip_fail(e, "shift up");
      if (l == L - 1 && fork2 && op->sched_il == 2) {
        pie_status ps = fork_translate();
        if (ps) return ps;
      }
      if (perlev && l >= 4) {
        pie_status ps = fork_level(l);
        if (ps) return ps;
      }
    }
    if (oneset) {
      DevLevel lvs[24];
      const void* Ss[24];
      const void* Ts[24];
      void* Gs[24];
      const int n = L - 2;
      for (int i = 0; i < n; ++i) {
        lvs[i] = op->lv[3 + i];
        Ss[i] = op->dS[3 + i];
        Ts[i] = op->dTl[3 + i];
        Gs[i] = op->dG[3 + i];
      }
      if ((e = stage(op, PIE_STAGE_TRANSLATE, st, [&] {
             return launch_translate_levels<TF>(lvs, Ss, Ts, Gs, n, Q, R, st);
           })) != hipSuccess)
        return hip_fail(e, "translate");
    } else {
      for (int l = 3; l <= L; ++l)
        if (perlev ? l == 3 : (l < L || !fork2))
          if ((e = translate(l, st)) != hipSuccess) return hip_fail(e, "translate");
    }
    for (int l = 4; l <= L; ++l) {
      if (l == L && fork2) HIPCHK(hipStreamWaitEvent(st, op->ev_il, 0), "join");
      if (perlev) HIPCHK(hipStreamWaitEvent(st, op->ev_g[l], 0), "join");
      if ((e = stage(op, PIE_STAGE_SHIFT_DOWN, st, [&] {
             return launch_shift_down<TF>(op->lv[l], op->dG[l - 1], op->dG[l], op->dFl[l - 1], op->dPhl[l - 1],
                                          Q, R, op->force_ms, st);
           })) != hipSuccess)
        return hip_fail(e, "shift down");
    }
  }
  int rflags = (near ? 1 : 0) | (far ? 2 : 0) | (adj ? 4 : 0);
  if (fork) HIPCHK(hipStreamWaitEvent(st, op->ev_join, 0), "join");
  if ((e = stage(op, PIE_STAGE_RECEIVE, st, [&] {
         hipError_t e1 = launch_receive<TF, TN>(op->I, B, op->NJ, op->NT, op->lv[L].nb, op->maxinc, op->maxjoin,
                                                op->dG[L], op->dM, op->dAnti, Q, op->Qh, op->dPartJ, op->dPartT, R,
                                                rcap, rflags, y, ld, op->dPhi, st);
         if (e1 != hipSuccess) return e1;
         return launch_div_test(op->dCtri, op->dCs, op->dPhi, op->ne, R, y, ld, st);
       })) != hipSuccess)
    return hip_fail(e, "receive");
  return PIE_OK;
}

pie_status mvm(pie_op* op, const void* x, void* y, int64_t R, int flags, hipStream_t st) {
  // passes of at most pw columns; inside a pass the kernels take the
  // columns in register groups of 1, 2 or 4, and each column's arithmetic
  // is the same for any pass width or grouping
  int64_t r0 = 0;
  while (r0 < R) {
    const int w = (int)std::min<int64_t>(R - r0, op->pw);
    const void* xc = (const cx<double>*)x + r0;
    void* yc = (cx<double>*)y + r0;
    pie_status s;
    if (op->far_prec == PIE_FP32 && op->near_prec == PIE_FP32)
      s = mvm_chunk<float, float>(op, xc, yc, (int)R, w, flags, st);
    else if (op->far_prec == PIE_FP32)
      s = mvm_chunk<float, double>(op, xc, yc, (int)R, w, flags, st);
    else if (op->near_prec == PIE_FP32)
      s = mvm_chunk<double, float>(op, xc, yc, (int)R, w, flags, st);
    else
      s = mvm_chunk<double, double>(op, xc, yc, (int)R, w, flags, st);
    if (s) return s;
    r0 += w;
  }
  return PIE_OK;
}

pie_status check_op_call(const pie_op* op, const void* x, const void* y, int64_t R) {
  if (!op || !x || !y) {
    set_error("null operator or vector");
    return PIE_ERR_ARG;
  }
  if (R < 1 || R > op->max_rhs) {
    set_error("R must be in [1, max_rhs]");
    return PIE_ERR_ARG;
  }
  if (x == y) {
    set_error("x and y must not overlap");
    return PIE_ERR_ARG;
  }
  return PIE_OK;
}

}  // namespace

// =========================================================================
// C ABI
// =========================================================================
extern "C" {

size_t pie_last_error(char* buf, size_t len) {
  const std::string& s = pie::g_err;
  if (buf && len) {
    size_t n = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return s.size();
}

int32_t pie_version(void) { return 100; }

pie_status pie_mesh_create(const double* V, int64_t nv, const int32_t* T, int64_t nt, pie_mesh** out) {
  if (!out) {
    pie::set_error("null output handle");
    return PIE_ERR_ARG;
  }
  *out = nullptr;
  auto h = std::make_unique<pie_mesh>();
  pie_status s = pie::build_mesh(V, nv, T, nt, h->m);
  if (s) return s;
  *out = h.release();
  return PIE_OK;
}
void pie_mesh_destroy(pie_mesh* m) { delete m; }

pie_status pie_mesh_icosphere(int32_t subdiv, double radius, double jitter, uint64_t seed, pie_mesh** out) {
  if (!out) {
    pie::set_error("null output handle");
    return PIE_ERR_ARG;
  }
  *out = nullptr;
  std::vector<double> V;
  std::vector<int32_t> T;
  pie_status s = pie::icosphere(subdiv, radius, jitter, seed, V, T);
  if (s) return s;
  return pie_mesh_create(V.data(), (int64_t)V.size() / 3, T.data(), (int64_t)T.size() / 3, out);
}

pie_status pie_mesh_geometry(const pie_mesh* m, int64_t* nv, int64_t* nt, double* V, int32_t* T) {
  if (!m) {
    pie::set_error("null mesh");
    return PIE_ERR_ARG;
  }
  if (nv) *nv = m->m.nv;
  if (nt) *nt = m->m.nt;
  if (V) std::memcpy(V, m->m.V.data(), m->m.V.size() * sizeof(double));
  if (T) std::memcpy(T, m->m.T.data(), m->m.T.size() * sizeof(int32_t));
  return PIE_OK;
}

pie_status pie_mesh_sizes(const pie_mesh* m, int64_t* nE, int64_t* nT) {
  if (!m) {
    pie::set_error("null mesh");
    return PIE_ERR_ARG;
  }
  if (nE) *nE = m->m.ne;
  if (nT) *nT = m->m.nt;
  return PIE_OK;
}

pie_status pie_mesh_edges(const pie_mesh* m, int32_t* edges, int32_t* tri, int32_t* free_vertex) {
  if (!m) {
    pie::set_error("null mesh");
    return PIE_ERR_ARG;
  }
  size_t n = 2 * (size_t)m->m.ne;
  if (edges) std::memcpy(edges, m->m.edge.data(), n * sizeof(int32_t));
  if (tri) std::memcpy(tri, m->m.etri.data(), n * sizeof(int32_t));
  if (free_vertex) std::memcpy(free_vertex, m->m.efree.data(), n * sizeof(int32_t));
  return PIE_OK;
}

pie_status pie_tree_build(const pie_mesh* m, int32_t levels, pie_tree** out) {
  if (!m || !out) {
    pie::set_error("null mesh or output handle");
    return PIE_ERR_ARG;
  }
  *out = nullptr;
  auto h = std::make_unique<pie_tree>();
  pie_status s = pie::build_tree(m->m, levels, h->t);
  if (s) return s;
  *out = h.release();
  return PIE_OK;
}
void pie_tree_destroy(pie_tree* t) { delete t; }

pie_status pie_tree_query(const pie_tree* th, int32_t what, int32_t level, int64_t* count, int64_t* data) {
  if (!th || !count) {
    pie::set_error("null tree or count");
    return PIE_ERR_ARG;
  }
  const pie::Tree& t = th->t;
  const std::vector<int64_t>* v = nullptr;
  bool needs_level = what == PIE_TQ_NBOX || what == PIE_TQ_COORDS || what == PIE_TQ_PARENT ||
                     what == PIE_TQ_IL_PTR || what == PIE_TQ_IL_SRC || what == PIE_TQ_IL_OFF;
  if (needs_level && (level < 1 || level > t.L)) {
    pie::set_error("level out of range");
    return PIE_ERR_ARG;
  }
  if ((what == PIE_TQ_IL_PTR || what == PIE_TQ_IL_SRC || what == PIE_TQ_IL_OFF) && level < 3) {
    pie::set_error("interaction lists exist for levels >= 3");
    return PIE_ERR_ARG;
  }
  switch (what) {
    case PIE_TQ_NBOX:
      *count = t.lev[level].nb;
      return PIE_OK;
    case PIE_TQ_COORDS: v = &t.lev[level].coords; break;
    case PIE_TQ_PARENT: v = &t.lev[level].parent; break;
    case PIE_TQ_PERM: v = &t.perm; break;
    case PIE_TQ_BOXPTR: v = &t.box_ptr; break;
    case PIE_TQ_NEAR_PTR: v = &t.near_ptr; break;
    case PIE_TQ_NEAR_IDX: v = &t.near_idx; break;
    case PIE_TQ_IL_PTR: v = &t.lev[level].il_ptr; break;
    case PIE_TQ_IL_SRC: v = &t.lev[level].il_src; break;
    case PIE_TQ_IL_OFF: v = &t.lev[level].il_off; break;
    default:
      pie::set_error("unknown tree query");
      return PIE_ERR_ARG;
  }
  *count = (int64_t)v->size();
  if (data && !v->empty()) std::memcpy(data, v->data(), v->size() * sizeof(int64_t));
  return PIE_OK;
}

void pie_options_default(pie_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->version = 1;
  o->near_prec = PIE_FP64;
  o->far_prec = PIE_FP64;
  o->max_rhs = 1;
}

pie_status pie_operator_create(const pie_mesh* m, const pie_tree* t, double freq_hz, const pie_options* opt,
                               void* stream, pie_op** out) {
  if (!m || !t || !opt || !out) {
    pie::set_error("null argument");
    return PIE_ERR_ARG;
  }
  *out = nullptr;
  if (opt->version != 1) {
    pie::set_error("pie_options.version must be 1");
    return PIE_ERR_ARG;
  }
  if (!(freq_hz > 0.0) || !std::isfinite(freq_hz)) {
    pie::set_error("frequency must be positive and finite");
    return PIE_ERR_ARG;
  }
  if ((opt->near_prec != PIE_FP32 && opt->near_prec != PIE_FP64) ||
      (opt->far_prec != PIE_FP32 && opt->far_prec != PIE_FP64)) {
    pie::set_error("precision must be PIE_FP32 or PIE_FP64");
    return PIE_ERR_ARG;
  }
  if (opt->flags & ~PIE_OPT_MATRIX_SHIFTS) {
    pie::set_error("unknown pie_options.flags bits");
    return PIE_ERR_ARG;
  }
  if (opt->max_rhs < 1 || opt->max_rhs > 4096) {
    pie::set_error("max_rhs must be in [1, 4096]");
    return PIE_ERR_ARG;
  }
  if (t->t.mesh != &m->m) {
    pie::set_error("tree was built for a different mesh");
    return PIE_ERR_ARG;
  }
  auto op = std::make_unique<pie_op>();
  op->mesh = &m->m;
  op->tree = &t->t;
  op->freq = freq_hz;
  op->omega = 2.0 * pie::kPi * freq_hz;
  op->k = op->omega / pie::kC0;
  op->w2e = op->omega * op->omega * pie::kEps0;
  op->near_prec = opt->near_prec;
  op->far_prec = opt->far_prec;
  const bool f32 = opt->far_prec == PIE_FP32;
  // FP64 far field: x = 0.08 keeps the translation's rounding nonlinearity
  // near 4e-6; deeper trees accumulate more of the inter-level rescaling
  // error (proportional to x^2), so 6 levels take 0.07 and 7 or more 0.06
  // (nonlinearity 1e-5 and 3e-5)
  const int Lt = t->t.L;
  op->xs = opt->x > 0.0 ? opt->x : (f32 ? 0.15 : (Lt <= 5 ? 0.08 : (Lt == 6 ? 0.07 : 0.06)));
  // truncation number of Eq. (5) per level from the level's box size k d_l:
  // tau = 7 up to k d = 0.8, 8 up to 1.6, 9 up to 3.2, 10 up to 4.8 (FP64
  // default; measured against sampled dense rows at 1 to 3 wavelengths), or
  // the caller's tau at every level; the k-space samples are those of the
  // largest tau, at every level
  op->tau_l.assign(Lt + 1, 0);
  int tmax = 0;
  for (int l = 3; l <= Lt; ++l) {
    const double kd = op->k * t->t.side / (double)(int64_t(1) << (l - 1));
    const int tl = opt->tau > 0 ? opt->tau : (f32 ? 4 : (kd <= 0.8 ? 7 : (kd <= 1.6 ? 8 : (kd <= 3.2 ? 9 : 10))));
    const double kdmax = f32 || tl < 7 ? 1.0 : (tl < 9 ? 1.6 : (tl < 10 ? 3.2 : 4.8));
    if (kd > kdmax) {
      pie::set_error("level-" + std::to_string(l) + " boxes (k d = " + std::to_string(kd) +
                     ") exceed what the truncation number covers: use more levels, or the FP64 far field");
      return PIE_ERR_UNSUPPORTED;
    }
    op->tau_l[l] = tl;
    tmax = std::max(tmax, tl);
  }
  op->tau = tmax;
  op->nth = opt->n_theta > 0 ? opt->n_theta : op->tau + 1;
  op->nph = opt->n_phi > 0 ? opt->n_phi : 2 * op->tau + 2;
  op->Q = op->nth * op->nph;
  op->max_rhs = opt->max_rhs;
  op->force_ms = (opt->flags & PIE_OPT_MATRIX_SHIFTS) != 0;
  op->L = t->t.L;
  op->ne = (int)m->m.ne;
  op->nt = (int)m->m.nt;
  op->N = op->ne + op->nt;
  if (op->tau > 20 || op->Q > 1024 || (op->nph & 1)) {
    pie::set_error("tau <= 20, Q <= 1024 and an even n_phi are required");
    return PIE_ERR_ARG;
  }
  // round-off amplification of the sampled translation at level l:
  // (2 tau_l + 1)!!/(2 x_l)^tau_l with x_l = k d_l / s_l = max(k d_l, x)
  double amp = 0.0;
  for (int l = 3; l <= Lt; ++l) {
    const double kd = op->k * t->t.side / (double)(int64_t(1) << (l - 1));
    amp = std::max(amp, dfact(2 * op->tau_l[l] + 1) / std::pow(2.0 * std::max(kd, op->xs), op->tau_l[l]));
  }
  const double eps = f32 ? 5.96e-8 : 1.11e-16;
  if (eps * amp > 1e-2) {
    pie::set_error("tau and x amplify round-off beyond 1e-2 in this far-field precision");
    return PIE_ERR_PRECISION;
  }
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipGetDevice(&op->device), "hipGetDevice");
  HIPCHK(hipStreamCreateWithFlags(&op->side, hipStreamNonBlocking), "side stream");
  HIPCHK(hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming), "fork event");
  HIPCHK(hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming), "join event");
  HIPCHK(hipStreamCreateWithFlags(&op->side2, hipStreamNonBlocking), "side stream");
  op->il_st.assign(op->L + 1, nullptr);
  op->ev_s.assign(op->L + 1, nullptr);
  op->ev_g.assign(op->L + 1, nullptr);
  for (int l = 4; l <= op->L; ++l) {
    HIPCHK(hipStreamCreateWithFlags(&op->il_st[l], hipStreamNonBlocking), "level stream");
    HIPCHK(hipEventCreateWithFlags(&op->ev_s[l], hipEventDisableTiming), "fork event");
    HIPCHK(hipEventCreateWithFlags(&op->ev_g[l], hipEventDisableTiming), "join event");
  }
  HIPCHK(hipEventCreateWithFlags(&op->ev_agg, hipEventDisableTiming), "fork event");
  HIPCHK(hipEventCreateWithFlags(&op->ev_il, hipEventDisableTiming), "join event");
  pie_status s = build_operator(op.get(), st);
  if (s) return s;
  *out = op.release();
  return PIE_OK;
}

void pie_operator_destroy(pie_op* op) { delete op; }

pie_status pie_operator_info(const pie_op* op, int32_t what, int64_t* value) {
  if (!op || !value) {
    pie::set_error("null argument");
    return PIE_ERR_ARG;
  }
  switch (what) {
    case PIE_OI_N: *value = op->N; break;
    case PIE_OI_Q: *value = op->Q; break;
    case PIE_OI_TAU: *value = op->tau; break;
    case PIE_OI_NEAR_BLOCKS: *value = op->NJ.nblk + op->NT.nblk; break;
    case PIE_OI_NEAR_ENTRIES: *value = op->near_entries; break;
    case PIE_OI_NEAR_BYTES: *value = op->near_entries * (op->near_prec == PIE_FP32 ? 8 : 16); break;
    case PIE_OI_NBOX_FINEST: *value = op->lv[op->L].nb; break;
    case PIE_OI_IL_PAIRS: *value = op->il_pairs; break;
    case PIE_OI_INCIDENCES: *value = op->ninc; break;
    case PIE_OI_DEVICE_BYTES: *value = (int64_t)op->bytes; break;
    case PIE_OI_NEAR_ENTRIES_RWG: *value = op->near_entries_J; break;
    case PIE_OI_NEAR_ENTRIES_TRI: *value = op->near_entries_T; break;
    default:
      if (what >= PIE_OI_TAU_LEVEL(3) && what <= PIE_OI_TAU_LEVEL(op->L)) {
        *value = op->tau_l[what - PIE_OI_TAU_LEVEL(0)];
        break;
      }
      pie::set_error("unknown operator query");
      return PIE_ERR_ARG;
  }
  return PIE_OK;
}

pie_status pie_operator_level(const pie_op* op, int32_t level, double* s, double* kappa, double* box_side) {
  if (!op || level < 3 || level > op->L) {
    pie::set_error("null operator or level out of range");
    return PIE_ERR_ARG;
  }
  if (s) *s = op->s_l[level];
  if (kappa) *kappa = op->kappa_l[level];
  if (box_side) *box_side = op->d_l[level];
  return PIE_OK;
}

pie_status pie_matvec(pie_op* op, const void* x, void* y, int64_t R, int32_t adjoint, void* stream) {
  pie_status s = check_op_call(op, x, y, R);
  if (s) return s;
  return mvm(op, x, y, R, 3 | (adjoint ? 4 : 0), (hipStream_t)stream);
}

pie_status pie_matvec_near(pie_op* op, const void* x, void* y, int64_t R, void* stream) {
  pie_status s = check_op_call(op, x, y, R);
  if (s) return s;
  return mvm(op, x, y, R, 1, (hipStream_t)stream);
}

pie_status pie_matvec_far(pie_op* op, const void* x, void* y, int64_t R, void* stream) {
  pie_status s = check_op_call(op, x, y, R);
  if (s) return s;
  return mvm(op, x, y, R, 2, (hipStream_t)stream);
}

pie_status pie_schedule_get(const pie_op* op, pie_schedule* out) {
  if (!op || !out) {
    pie::set_error("null operator or output");
    return PIE_ERR_ARG;
  }
  *out = pie_schedule{1, op->sched_near, op->sched_il, op->sched_chunk};
  return PIE_OK;
}

pie_status pie_schedule_set(pie_op* op, const pie_schedule* sch) {
  if (!op || !sch || sch->version != 1) {
    pie::set_error("null operator or schedule, or schedule version != 1");
    return PIE_ERR_ARG;
  }
  if (sch->near_fork < PIE_NEAR_SERIAL || sch->near_fork > PIE_NEAR_FORK_AFTER_AGGREGATE ||
      (sch->il_fork < 0 || sch->il_fork > 4) ||
      (sch->max_chunk != 1 && sch->max_chunk != 2 && sch->max_chunk != 4)) {
    pie::set_error("invalid schedule");
    return PIE_ERR_ARG;
  }
  op->sched_near = sch->near_fork;
  op->sched_il = sch->il_fork;
  op->sched_chunk = sch->max_chunk;
  return PIE_OK;
}

pie_status pie_autotune(pie_op* op, const void* x, void* y, int64_t R, int32_t reps, void* stream,
                        pie_schedule* chosen, double* ms) {
  pie_status s = check_op_call(op, x, y, R);
  if (s) return s;
  if (reps < 1 || op->prof) {
    pie::set_error(reps < 1 ? "reps must be >= 1" : "stage profiling must be off while tuning");
    return PIE_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0), "tuner event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    pie::set_error("tuner event");
    return PIE_ERR_HIP;
  }
  pie_schedule best{1, op->sched_near, op->sched_il, op->sched_chunk};
  double best_ms = 1e300;
  s = PIE_OK;
  std::vector<pie_schedule> cand;
  for (int nf = PIE_NEAR_SERIAL; nf <= PIE_NEAR_FORK_AFTER_AGGREGATE; ++nf)
    for (int il = 0; il <= 4; ++il)
      for (int ch : {4, 2, 1})
        // register groups wider than R or than the operator's limit repeat a narrower one
        if (ch == 1 || (ch <= op->rc && ch <= R)) cand.push_back(pie_schedule{1, nf, il, ch});
  // two rounds over the candidates, each keeping its faster round, so that
  // the order of measurement does not favour any schedule
  std::vector<double> t_ms(cand.size(), 1e300);
  for (int round = 0; round < 2 && !s; ++round)
    for (size_t c = 0; c < cand.size() && !s; ++c) {
      op->sched_near = cand[c].near_fork;
      op->sched_il = cand[c].il_fork;
      op->sched_chunk = cand[c].max_chunk;
      if ((s = mvm(op, x, y, R, 3, st))) break;
      if (hipEventRecord(e0, st) != hipSuccess) { s = PIE_ERR_HIP; break; }
      for (int i = 0; i < reps && !s; ++i) s = mvm(op, x, y, R, 3, st);
      if (s) break;
      float t = 0.0f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
        s = PIE_ERR_HIP;
        break;
      }
      t_ms[c] = std::min(t_ms[c], (double)t / reps);
    }
  for (size_t c = 0; c < cand.size(); ++c)
    if (t_ms[c] < best_ms) {
      best_ms = t_ms[c];
      best = cand[c];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  op->sched_near = best.near_fork;
  op->sched_il = best.il_fork;
  op->sched_chunk = best.max_chunk;
  if (s) {
    if (s == PIE_ERR_HIP) pie::set_error("tuner timing failed");
    return s;
  }
  if (chosen) *chosen = best;
  if (ms) *ms = best_ms;
  return PIE_OK;
}

pie_status pie_graph_create(pie_op* op, const void* x, void* y, int64_t R, int32_t adjoint, pie_graph** out) {
  if (!out) {
    pie::set_error("null output handle");
    return PIE_ERR_ARG;
  }
  *out = nullptr;
  pie_status s = check_op_call(op, x, y, R);
  if (s) return s;
  if (op->prof) {
    pie::set_error("stage profiling must be off while capturing");
    return PIE_ERR_ARG;
  }
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
  auto g = std::make_unique<pie_graph>();
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    s = mvm(op, x, y, R, 3 | (adjoint ? 4 : 0), cs);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &gr);
    g->graph = gr;
    if (!s && e2 != hipSuccess) e = e2;
    if (!s && e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  }
  (void)hipStreamDestroy(cs);
  if (s) return s;
  if (e != hipSuccess) return hip_fail(e, "graph capture");
  *out = g.release();
  return PIE_OK;
}

pie_status pie_graph_create_batch(pie_op* const* ops, int32_t nobj, const void* const* xs, void* const* ys,
                                  const int64_t* Rs, int32_t adjoint, pie_graph** out) {
  if (!out || !ops || !xs || !ys || !Rs || nobj < 1) {
    pie::set_error("null argument or empty batch");
    return PIE_ERR_ARG;
  }
  *out = nullptr;
  for (int i = 0; i < nobj; ++i) {
    pie_status s = check_op_call(ops[i], xs[i], ys[i], Rs[i]);
    if (s) return s;
    if (ops[i]->prof) {
      pie::set_error("stage profiling must be off while capturing");
      return PIE_ERR_ARG;
    }
    for (int j = 0; j < i; ++j)
      if (ops[j] == ops[i]) {
        pie::set_error("an operator appears twice in the batch");
        return PIE_ERR_ARG;
      }
  }
  // the objects' MVMs are captured one after another on one private stream
  // (each with its own side-stream forks and joins, as in pie_graph_create)
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
  auto g = std::make_unique<pie_graph>();
  pie_status s = PIE_OK;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int i = 0; i < nobj && !s; ++i) s = mvm(ops[i], xs[i], ys[i], Rs[i], 3 | (adjoint ? 4 : 0), cs);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &gr);
    g->graph = gr;
    if (!s && e2 != hipSuccess) e = e2;
    if (!s && e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  }
  (void)hipStreamDestroy(cs);
  if (s) return s;
  if (e != hipSuccess) return hip_fail(e, "batch graph capture");
  *out = g.release();
  return PIE_OK;
}

pie_status pie_batch_create(pie_op* const* ops, int32_t nobj, pie_batch** out) {
  if (!out || !ops || nobj < 1) {
    pie::set_error("null argument or empty batch");
    return PIE_ERR_ARG;
  }
  *out = nullptr;
  for (int i = 0; i < nobj; ++i) {
    if (!ops[i]) {
      pie::set_error("null operator in the batch");
      return PIE_ERR_ARG;
    }
    for (int j = 0; j < i; ++j)
      if (ops[j] == ops[i]) {
        pie::set_error("an operator appears twice in the batch");
        return PIE_ERR_ARG;
      }
  }
  auto b = std::make_unique<pie_batch>();
  b->ops.assign(ops, ops + nobj);
  HIPCHK(hipEventCreateWithFlags(&b->start, hipEventDisableTiming), "batch event");
  for (int i = 0; i < nobj; ++i) {
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "batch stream");
    b->st.push_back(s);
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming), "batch event");
    b->done.push_back(e);
  }
  *out = b.release();
  return PIE_OK;
}

pie_status pie_batch_matvec(pie_batch* b, const void* const* xs, void* const* ys, const int64_t* Rs,
                            int32_t adjoint, void* stream) {
  if (!b || !xs || !ys || !Rs) {
    pie::set_error("null argument");
    return PIE_ERR_ARG;
  }
  const int n = (int)b->ops.size();
  for (int i = 0; i < n; ++i) {
    pie_status s = check_op_call(b->ops[i], xs[i], ys[i], Rs[i]);
    if (s) return s;
    if (b->ops[i]->prof) {
      pie::set_error("stage profiling must be off for a batch call");
      return PIE_ERR_ARG;
    }
  }
  hipStream_t cs = (hipStream_t)stream;
  HIPCHK(hipEventRecord(b->start, cs), "batch fork");
  for (int i = 0; i < n; ++i) {
    HIPCHK(hipStreamWaitEvent(b->st[i], b->start, 0), "batch fork");
    pie_status s = mvm(b->ops[i], xs[i], ys[i], Rs[i], 3 | (adjoint ? 4 : 0), b->st[i]);
    if (s) return s;
    HIPCHK(hipEventRecord(b->done[i], b->st[i]), "batch join");
    HIPCHK(hipStreamWaitEvent(cs, b->done[i], 0), "batch join");
  }
  return PIE_OK;
}

void pie_batch_destroy(pie_batch* b) { delete b; }

pie_status pie_graph_launch(pie_graph* g, void* stream) {
  if (!g || !g->exec) {
    pie::set_error("null graph");
    return PIE_ERR_ARG;
  }
  HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)stream), "graph launch");
  return PIE_OK;
}

void pie_graph_destroy(pie_graph* g) { delete g; }

pie_status pie_profile_enable(pie_op* op, int32_t on) {
  if (!op) {
    pie::set_error("null operator");
    return PIE_ERR_ARG;
  }
  for (auto& u : op->ev_used) {
    op->ev_pool.push_back(u.second.first);
    op->ev_pool.push_back(u.second.second);
  }
  op->ev_used.clear();
  op->prof = on != 0;
  return PIE_OK;
}

pie_status pie_profile_read(pie_op* op, double* ms, int64_t* launches) {
  if (!op) {
    pie::set_error("null operator");
    return PIE_ERR_ARG;
  }
  double acc[PIE_NSTAGES] = {0};
  int64_t cnt[PIE_NSTAGES] = {0};
  for (auto& u : op->ev_used) {
    HIPCHK(hipEventSynchronize(u.second.second), "profile sync");
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, u.second.first, u.second.second), "profile elapsed");
    acc[u.first] += t;
    cnt[u.first] += 1;
  }
  for (int i = 0; i < PIE_NSTAGES; ++i) {
    if (ms) ms[i] = acc[i];
    if (launches) launches[i] = cnt[i];
  }
  return PIE_OK;
}

pie_status pie_rhs_planewave(pie_op* op, int64_t R, const double* khat, const double* pol, const double* amp,
                             int32_t gauge, void* b, void* stream) {
  if (!op || !khat || !pol || !amp || !b) {
    pie::set_error("null argument");
    return PIE_ERR_ARG;
  }
  if (R < 1 || R > op->max_rhs || (gauge != 0 && gauge != 1)) {
    pie::set_error("R must be in [1, max_rhs] and gauge 0 or 1");
    return PIE_ERR_ARG;
  }
  for (int64_t i = 0; i < 3 * R; ++i)
    if (!std::isfinite(khat[i]) || !std::isfinite(pol[i])) {
      pie::set_error("non-finite plane-wave direction or polarisation");
      return PIE_ERR_NONFINITE;
    }
  for (int64_t i = 0; i < 2 * R; ++i)
    if (!std::isfinite(amp[i])) {
      pie::set_error("non-finite amplitude");
      return PIE_ERR_NONFINITE;
    }
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(op->dKhR, khat, 3 * R * sizeof(double), hipMemcpyHostToDevice, st), "rhs copy");
  HIPCHK(hipMemcpyAsync(op->dPolR, pol, 3 * R * sizeof(double), hipMemcpyHostToDevice, st), "rhs copy");
  HIPCHK(hipMemcpyAsync(op->dAmpR, amp, 2 * R * sizeof(double), hipMemcpyHostToDevice, st), "rhs copy");
  hipError_t e = pie::launch_rhs(geo(op), op->dCs, op->dCtri, op->dCfv, op->ne, op->nt, op->dKhR, op->dPolR,
                                 op->dAmpR, (int)R, gauge, op->k, op->omega, b, st);
  if (e != hipSuccess) return hip_fail(e, "rhs");
  HIPCHK(hipStreamSynchronize(st), "rhs");  // host arrays are released on return
  return PIE_OK;
}

pie_status pie_farfield(pie_op* op, const void* x, int64_t R, const double* dirs, int64_t nd, void* F,
                        void* stream) {
  if (!op || !x || !dirs || !F || nd < 1) {
    pie::set_error("null argument or no directions");
    return PIE_ERR_ARG;
  }
  if (R < 1 || R > op->max_rhs) {
    pie::set_error("R must be in [1, max_rhs]");
    return PIE_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  if (nd > op->ndirs_cap) {
    pie_status s = dalloc(op, &op->dDirs, 3 * (size_t)nd);
    if (s) return s;
    op->ndirs_cap = nd;
  }
  HIPCHK(hipMemcpyAsync(op->dDirs, dirs, 3 * nd * sizeof(double), hipMemcpyHostToDevice, st), "dirs copy");
  hipError_t e = pie::launch_farfield(geo(op), op->dCs, op->dCtri, op->dCfv, op->ne, x, (int)R, op->dDirs, (int)nd,
                                      op->k, op->omega, F, st);
  if (e != hipSuccess) return hip_fail(e, "farfield");
  HIPCHK(hipStreamSynchronize(st), "farfield");
  return PIE_OK;
}

pie_status pie_farfield_adjoint(pie_op* op, const void* gF, int64_t R, const double* dirs, int64_t nd, void* gx,
                                void* stream) {
  if (!op || !gF || !dirs || !gx || nd < 1) {
    pie::set_error("null argument or no directions");
    return PIE_ERR_ARG;
  }
  if (R < 1 || R > op->max_rhs) {
    pie::set_error("R must be in [1, max_rhs]");
    return PIE_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  if (nd > op->ndirs_cap) {
    pie_status s = dalloc(op, &op->dDirs, 3 * (size_t)nd);
    if (s) return s;
    op->ndirs_cap = nd;
  }
  HIPCHK(hipMemcpyAsync(op->dDirs, dirs, 3 * nd * sizeof(double), hipMemcpyHostToDevice, st), "dirs copy");
  hipError_t e = pie::launch_farfield_adj(geo(op), op->dCs, op->dCtri, op->dCfv, op->ne, op->nt, gF, (int)R,
                                          op->dDirs, (int)nd, op->k, op->omega, gx, st);
  if (e != hipSuccess) return hip_fail(e, "farfield adjoint");
  HIPCHK(hipStreamSynchronize(st), "farfield adjoint");
  return PIE_OK;
}

void pie_solve_opts_default(pie_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->version = 2;
  o->restart = 100;
  o->maxit = 1000;
  o->refine = 1;
  o->tol = 1e-6;
  o->inner_tol = 0.0;
}

}  // extern "C"

// ------------------------------------------------------------------ GMRES --
namespace {

// GMRES(m) with CGS2 on the equilibrated operator D Z D for all R columns in
// lock step; each column keeps its own Hessenberg matrix and rotations and is
// frozen once its residual estimate meets tol.  xhat (device) is updated.
// Block-diagonal preconditioner: the finest boxes' self blocks Z_bb in FP64
// (computed on the device with the near-field entry routine), inverted on
// the host by Gauss-Jordan elimination with partial pivoting, stored back in
// place.  Z^H = conj(Z) (Z is symmetric), so the adjoint solve uses the
// same blocks through its conjugated input and output.
pie_status build_prec(pie_op* op) {
  const pie::Tree& t = *op->tree;
  const int L = op->L;
  const int nbox = (int)t.lev[L].nb;
  std::vector<int64_t> off(nbox + 1, 0);
  for (int b = 0; b < nbox; ++b) {
    const int64_t nb = (int64_t)(t.box_ptr[b + 1] - t.box_ptr[b]);
    off[b + 1] = off[b] + nb * nb;
  }
  cx<double>* blocks;
  int64_t* doff;
  pie_status s;
  if ((s = dalloc(op, &blocks, (size_t)off[nbox])) || (s = dalloc(op, &doff, (size_t)nbox + 1))) return s;
  HIPCHK(hipMemcpy(doff, off.data(), (nbox + 1) * sizeof(int64_t), hipMemcpyHostToDevice), "prec offsets");
  hipError_t e = launch_diag_blocks(geo(op), basis(op), op->dBoxPtr, doff, nbox, blocks, op->k, op->w2e, nullptr);
  if (e != hipSuccess) return hip_fail(e, "self blocks");
  HIPCHK(hipDeviceSynchronize(), "self blocks");
  std::vector<std::complex<double>> h((size_t)off[nbox]);
  HIPCHK(hipMemcpy(h.data(), blocks, h.size() * 16, hipMemcpyDeviceToHost), "self blocks copy");
  // Gauss-Jordan [M | I] -> [I | M^-1] with row pivoting, box b of
  // [b0, nbox) in steps of `step`; false on a singular block
  auto invert = [&](int b0, int step) {
    std::vector<std::complex<double>> a;
    for (int b = b0; b < nbox; b += step) {
      const int n = (int)(t.box_ptr[b + 1] - t.box_ptr[b]);
      std::complex<double>* M = h.data() + off[b];
      a.assign((size_t)n * 2 * n, 0.0);
      for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) a[(size_t)i * 2 * n + j] = M[(size_t)i * n + j];
        a[(size_t)i * 2 * n + n + i] = 1.0;
      }
      for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
          if (std::abs(a[(size_t)i * 2 * n + c]) > std::abs(a[(size_t)p * 2 * n + c])) p = i;
        if (!(std::abs(a[(size_t)p * 2 * n + c]) > 0.0)) return false;
        if (p != c)
          for (int j = 0; j < 2 * n; ++j) std::swap(a[(size_t)p * 2 * n + j], a[(size_t)c * 2 * n + j]);
        const std::complex<double> inv = 1.0 / a[(size_t)c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) a[(size_t)c * 2 * n + j] *= inv;
        for (int i = 0; i < n; ++i) {
          if (i == c) continue;
          const std::complex<double> f = a[(size_t)i * 2 * n + c];
          if (f == 0.0) continue;
          for (int j = 0; j < 2 * n; ++j) a[(size_t)i * 2 * n + j] -= f * a[(size_t)c * 2 * n + j];
        }
      }
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) M[(size_t)i * n + j] = a[(size_t)i * 2 * n + n + j];
    }
    return true;
  };
  // boxes are independent: strided over up to 16 host threads
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<char> ok(nth, 1);
  {
    std::vector<std::thread> pool;
    for (int i = 1; i < nth; ++i) pool.emplace_back([&, i] { ok[i] = invert(i, nth); });
    ok[0] = invert(0, nth);
    for (auto& th : pool) th.join();
  }
  for (char o : ok)
    if (!o) {
      set_error("singular self block of a finest box (preconditioner)");
      return PIE_ERR_UNSUPPORTED;
    }
  HIPCHK(hipMemcpy(blocks, h.data(), h.size() * 16, hipMemcpyHostToDevice), "preconditioner copy");
  op->dPrec = blocks;
  op->dPrecOff = doff;
  return PIE_OK;
}

// The operator of a solve: mvm flags (3 = near + far, 4 = adjoint) plus
// SOLVE_PULSE_BLOCK, which applies the pulse-pulse block alone, embedded as
// diag(0, Z^AA): the RWG rows of the input are cleared before the product
// and those of the output after it, so a right-hand side without RWG rows
// keeps every Krylov vector in the pulse rows.
constexpr int SOLVE_PULSE_BLOCK = 8;
pie_status solve_mvm(pie_op* op, cx<double>* x, cx<double>* y, int64_t R, int flags, hipStream_t st) {
  const size_t nj = (size_t)op->ne * R * sizeof(cx<double>);
  if (flags & SOLVE_PULSE_BLOCK) HIPCHK(hipMemsetAsync(x, 0, nj, st), "clear RWG rows");
  pie_status s = mvm(op, x, y, R, flags & 7, st);
  if (s) return s;
  if (flags & SOLVE_PULSE_BLOCK) HIPCHK(hipMemsetAsync(y, 0, nj, st), "clear RWG rows");
  return PIE_OK;
}

pie_status gmres_equilibrated(pie_op* op, const cx<double>* rhat, cx<double>* xhat, int R, const pie_solve_opts& o,
                              double tol, int mflags, bool prec, int* iters, hipStream_t st, cx<double>* work) {
  // right preconditioning with P = D^-1 Minv D^-1 (Minv: inverses of the
  // finest boxes' self blocks): A P v = D Z (Minv D^-1 v), xhat += P V y
  const int nbox = (int)op->tree->lev[op->L].nb;
  const int N = op->N, m = std::max(1, o.restart);
  const size_t NR = (size_t)N * R;
  cx<double>* V = work;                    // (m+1) blocks
  cx<double>* w = V + (size_t)(m + 1) * NR;
  cx<double>* tmp = w + NR;
  cx<double>* dh = tmp + NR;               // (m+1) x R
  double* dn = (double*)(dh + (size_t)(m + 1) * R);
  std::vector<double> beta(R), nrm(R), inv(R), rhn(R);
  std::vector<std::complex<double>> H((size_t)R * (m + 1) * m), cs((size_t)R * m), sn((size_t)R * m),
      g((size_t)R * (m + 1)), h((size_t)(m + 1) * R), h2((size_t)(m + 1) * R);
  std::vector<int> kused(R, 0);
  std::vector<char> active(R, 1);
  hipError_t e;
  int total = 0;
  pie_status s;
  auto dots = [&](int nv, std::vector<std::complex<double>>& out) -> pie_status {
    if ((e = launch_dots(V, NR, nv, w, N, R, dh, st)) != hipSuccess) return hip_fail(e, "dots");
    HIPCHK(hipMemcpyAsync(out.data(), dh, (size_t)nv * R * 16, hipMemcpyDeviceToHost, st), "dots copy");
    HIPCHK(hipStreamSynchronize(st), "dots");
    return PIE_OK;
  };
  while (total < o.maxit) {
    // r = rhat - A xhat  (A = D Z D)
    if ((e = launch_scale_rows(xhat, op->dDiagScale, N, R, tmp, st)) != hipSuccess) return hip_fail(e, "scale");
    if ((s = solve_mvm(op, tmp, w, R, mflags, st))) return s;
    if ((e = launch_scale_rows(w, op->dDiagScale, N, R, w, st)) != hipSuccess) return hip_fail(e, "scale");
    if ((e = launch_sub(rhat, w, N, R, V, st)) != hipSuccess) return hip_fail(e, "sub");
    if ((e = launch_norms(V, N, R, dn, st)) != hipSuccess) return hip_fail(e, "norm");
    HIPCHK(hipMemcpyAsync(beta.data(), dn, R * 8, hipMemcpyDeviceToHost, st), "norm copy");
    if ((e = launch_norms(rhat, N, R, dn, st)) != hipSuccess) return hip_fail(e, "norm");
    HIPCHK(hipMemcpyAsync(nrm.data(), dn, R * 8, hipMemcpyDeviceToHost, st), "norm copy");
    HIPCHK(hipStreamSynchronize(st), "gmres");
    bool any = false;
    for (int r = 0; r < R; ++r) {
      rhn[r] = nrm[r];
      active[r] = beta[r] > tol * nrm[r];
      any = any || active[r];
      inv[r] = beta[r] > 0.0 ? 1.0 / beta[r] : 0.0;
      kused[r] = 0;
      for (int j = 0; j <= m; ++j) g[(size_t)r * (m + 1) + j] = 0.0;
      g[(size_t)r * (m + 1)] = beta[r];
    }
    if (!any) break;
    HIPCHK(hipMemcpyAsync(dn, inv.data(), R * 8, hipMemcpyHostToDevice, st), "inv copy");
    if ((e = launch_colscale(V, dn, N, R, st)) != hipSuccess) return hip_fail(e, "colscale");
    int j = 0;
    for (; j < m && total < o.maxit; ++j) {
      ++total;
      cx<double>* vj = V + (size_t)j * NR;
      e = prec ? launch_block_prec(vj, op->dDiagScale, op->dPrec, op->dPrecOff, op->dBoxPtr, op->dPerm, nbox, R,
                                   tmp, st)
               : launch_scale_rows(vj, op->dDiagScale, N, R, tmp, st);
      if (e != hipSuccess) return hip_fail(e, "scale");
      if ((s = solve_mvm(op, tmp, w, R, mflags, st))) return s;
      if ((e = launch_scale_rows(w, op->dDiagScale, N, R, w, st)) != hipSuccess) return hip_fail(e, "scale");
      // classical Gram-Schmidt, twice
      if ((s = dots(j + 1, h))) return s;
      HIPCHK(hipMemcpyAsync(dh, h.data(), (size_t)(j + 1) * R * 16, hipMemcpyHostToDevice, st), "h copy");
      if ((e = launch_update(w, V, NR, j + 1, dh, N, R, st)) != hipSuccess) return hip_fail(e, "update");
      if ((s = dots(j + 1, h2))) return s;
      HIPCHK(hipMemcpyAsync(dh, h2.data(), (size_t)(j + 1) * R * 16, hipMemcpyHostToDevice, st), "h copy");
      if ((e = launch_update(w, V, NR, j + 1, dh, N, R, st)) != hipSuccess) return hip_fail(e, "update");
      if ((e = launch_norms(w, N, R, dn, st)) != hipSuccess) return hip_fail(e, "norm");
      HIPCHK(hipMemcpyAsync(nrm.data(), dn, R * 8, hipMemcpyDeviceToHost, st), "norm copy");
      HIPCHK(hipStreamSynchronize(st), "gmres");
      bool any_active = false;
      for (int r = 0; r < R; ++r) {
        inv[r] = 0.0;
        if (!active[r]) continue;
        std::complex<double>* Hr = &H[(size_t)r * (m + 1) * m];
        for (int i = 0; i <= j; ++i) Hr[(size_t)i * m + j] = h[(size_t)i * R + r] + h2[(size_t)i * R + r];
        Hr[(size_t)(j + 1) * m + j] = nrm[r];
        // complex Givens rotations G_i = [[conj(c), conj(s)], [-s, c]] with
        // c = a / |(a, b)|, s = b / |(a, b)|, so that G_i (a, b) = (|(a, b)|, 0);
        // the same G_i is applied to later columns and to g
        for (int i = 0; i < j; ++i) {
          std::complex<double> c = cs[(size_t)r * m + i], sN = sn[(size_t)r * m + i];
          std::complex<double> a = Hr[(size_t)i * m + j], b = Hr[(size_t)(i + 1) * m + j];
          Hr[(size_t)i * m + j] = std::conj(c) * a + std::conj(sN) * b;
          Hr[(size_t)(i + 1) * m + j] = -sN * a + c * b;
        }
        std::complex<double> a = Hr[(size_t)j * m + j], b = Hr[(size_t)(j + 1) * m + j];
        double den = std::sqrt(std::norm(a) + std::norm(b));
        std::complex<double> c = den > 0 ? a / den : 1.0, sN = den > 0 ? b / den : 0.0;
        cs[(size_t)r * m + j] = c;
        sn[(size_t)r * m + j] = sN;
        Hr[(size_t)j * m + j] = den;
        Hr[(size_t)(j + 1) * m + j] = 0.0;
        std::complex<double>* gr = &g[(size_t)r * (m + 1)];
        gr[j + 1] = -sN * gr[j];
        gr[j] = std::conj(c) * gr[j];
        kused[r] = j + 1;
        active[r] = std::abs(gr[j + 1]) > tol * rhn[r];
        any_active = any_active || active[r];
        inv[r] = nrm[r] > 0.0 ? 1.0 / nrm[r] : 0.0;
      }
      cx<double>* vn = V + (size_t)(j + 1) * NR;
      HIPCHK(hipMemcpyAsync(vn, w, NR * 16, hipMemcpyDeviceToDevice, st), "copy");
      HIPCHK(hipMemcpyAsync(dn, inv.data(), R * 8, hipMemcpyHostToDevice, st), "inv copy");
      if ((e = launch_colscale(vn, dn, N, R, st)) != hipSuccess) return hip_fail(e, "colscale");
      // stop the cycle when every column meets tol relative to ||rhat||
      if (!any_active) break;
    }
    // y = H^-1 g per column; xhat += V y (the update kernel subtracts V h,
    // so h = -y is uploaded)
    std::vector<std::complex<double>> y((size_t)(m + 1) * R, 0.0);
    for (int r = 0; r < R; ++r) {
      int k = kused[r];
      std::complex<double>* Hr = &H[(size_t)r * (m + 1) * m];
      std::complex<double>* gr = &g[(size_t)r * (m + 1)];
      for (int i = k - 1; i >= 0; --i) {
        std::complex<double> acc = gr[i];
        for (int l = i + 1; l < k; ++l) acc -= Hr[(size_t)i * m + l] * y[(size_t)l * R + r];
        y[(size_t)i * R + r] = Hr[(size_t)i * m + i] != 0.0 ? acc / Hr[(size_t)i * m + i] : 0.0;
      }
    }
    for (auto& v : y) v = -v;
    int kmax = 0;
    for (int r = 0; r < R; ++r) kmax = std::max(kmax, kused[r]);
    if (kmax > 0) {
      HIPCHK(hipMemcpyAsync(dh, y.data(), (size_t)kmax * R * 16, hipMemcpyHostToDevice, st), "y copy");
      if (!prec) {
        if ((e = launch_update(xhat, V, NR, kmax, dh, N, R, st)) != hipSuccess) return hip_fail(e, "update");
      } else {
        // tmp = V y; w = Minv D^-1 tmp; xhat += D^-1 w
        HIPCHK(hipMemsetAsync(tmp, 0, NR * 16, st), "zero");
        if ((e = launch_update(tmp, V, NR, kmax, dh, N, R, st)) != hipSuccess) return hip_fail(e, "update");
        if ((e = launch_block_prec(tmp, op->dDiagScale, op->dPrec, op->dPrecOff, op->dBoxPtr, op->dPerm, nbox, R,
                                   w, st)) != hipSuccess)
          return hip_fail(e, "preconditioner");
        if ((e = launch_add_scaled(xhat, w, op->dDiagScale, N, R, st)) != hipSuccess) return hip_fail(e, "update");
      }
    }
    HIPCHK(hipStreamSynchronize(st), "gmres");
  }
  *iters = total;
  return PIE_OK;
}

}  // namespace

// Device workspace of a solve: the Krylov basis ((m + 1) N R), w and tmp,
// the Hessenberg column and norms, and four N R vectors of the refinement.
static size_t solve_workspace_bytes(int64_t N, int64_t R, int m) {
  const size_t NR = (size_t)N * R;
  return ((size_t)(m + 1) * NR + 2 * NR) * 16 + (size_t)(m + 1) * R * 16 + R * 16 + 4 * NR * 16;
}

// GMRES with outer refinement for Z x = b, or (block = SOLVE_PULSE_BLOCK)
// for the pulse-pulse block alone.
static pie_status solve_core(pie_op* op, pie_op* res_op, const void* b, void* x, int64_t R,
                             const pie_solve_opts* opts, pie_solve_info* info, void* stream, int block,
                             void* ws = nullptr, size_t ws_bytes = 0) {
  pie_status s = check_op_call(op, b, x, R);
  if (s) return s;
  pie_solve_opts o;
  pie_solve_opts_default(&o);
  if (opts) {
    if (opts->version == 1) {
      std::memcpy(&o, opts, offsetof(pie_solve_opts, precond));  // the fields of version 1
      o.version = 1;
      o.precond = 0;
    } else if (opts->version == 2) {
      o = *opts;
    } else {
      pie::set_error("pie_solve_opts.version must be 1 or 2");
      return PIE_ERR_ARG;
    }
  }
  if (o.restart < 1 || o.maxit < 1 || o.refine < 1 || !(o.tol > 0.0) || (o.precond != 0 && o.precond != 1)) {
    pie::set_error("restart, maxit, refine must be >= 1, tol > 0 and precond 0 or 1");
    return PIE_ERR_ARG;
  }
  const bool prec = o.precond == 1 && !block;
  if (prec && !op->dPrec && ws) {
    pie::set_error("the block-diagonal preconditioner is not built yet (building it allocates): call "
                   "pie_precond_apply or pie_solve with precond = 1 once first");
    return PIE_ERR_ARG;
  }
  if (prec && !op->dPrec && (s = build_prec(op))) return s;
  pie_op* rop = res_op ? res_op : op;
  if (rop->N != op->N || R > rop->max_rhs) {
    pie::set_error("residual operator does not match");
    return PIE_ERR_ARG;
  }
  const double inner = o.inner_tol > 0.0 ? o.inner_tol : o.tol;
  hipStream_t st = (hipStream_t)stream;
  const int N = op->N, m = o.restart;
  const size_t NR = (size_t)N * R;
  const size_t wbytes = solve_workspace_bytes(N, R, m);
  cx<double>* work = (cx<double>*)ws;
  std::unique_ptr<void, void (*)(void*)> guard(nullptr, [](void* p) { (void)hipFree(p); });
  if (work) {
    if (wbytes > ws_bytes) {
      pie::set_error("the solve needs " + std::to_string(wbytes) + " bytes of workspace (N R (restart + 7) 16 "
                     "+ small), more than the " + std::to_string(ws_bytes) + " bytes available");
      return PIE_ERR_ARG;
    }
  } else {
    HIPCHK(hipMalloc(&work, wbytes), "solver workspace");
    guard.reset(work);
  }
  cx<double>* rr = work + ((size_t)(m + 1) * NR + 2 * NR) + (size_t)(m + 1) * R + R;  // after solver area
  cx<double>* rhat = rr + NR;
  cx<double>* xh = rhat + NR;
  cx<double>* zx = xh + NR;
  double* dn = (double*)(work + (size_t)(m + 1) * NR + 2 * NR + (size_t)(m + 1) * R);
  cx<double>* X = (cx<double>*)x;
  hipError_t e;
  if (!o.use_x0) HIPCHK(hipMemsetAsync(X, 0, NR * 16, st), "zero x");
  // Residuals are measured in the equilibrated norm ||D v|| (D = diag
  // |Z_ii|^-1/2), the norm GMRES minimises: the rows of Eqs. (1) and (2)
  // carry different units, and at low frequency their scales differ by
  // orders of magnitude.  dnorm leaves D v in rhat.
  auto dnorm = [&](const void* v, std::vector<double>& out) -> pie_status {
    if ((e = pie::launch_scale_rows(v, op->dDiagScale, N, (int)R, rhat, st)) != hipSuccess)
      return hip_fail(e, "scale");
    if ((e = pie::launch_norms(rhat, N, (int)R, dn, st)) != hipSuccess) return hip_fail(e, "norm");
    HIPCHK(hipMemcpyAsync(out.data(), dn, R * 8, hipMemcpyDeviceToHost, st), "norm copy");
    HIPCHK(hipStreamSynchronize(st), "solve");
    return PIE_OK;
  };
  std::vector<double> bn(R), rn(R);
  if ((s = dnorm(b, bn))) return s;
  int iters = 0, refinements = 0;
  double relmax = 0.0;
  for (int k = 0; k < o.refine; ++k) {
    // residual with the residual operator
    if ((s = solve_mvm(rop, X, zx, R, 3 | (o.adjoint ? 4 : 0) | block, st))) return s;
    if ((e = pie::launch_sub(b, zx, N, (int)R, rr, st)) != hipSuccess) return hip_fail(e, "sub");
    if ((s = dnorm(rr, rn))) return s;  // rhat = D r
    relmax = 0.0;
    for (int r = 0; r < R; ++r) relmax = std::max(relmax, bn[r] > 0 ? rn[r] / bn[r] : 0.0);
    if (relmax <= o.tol) break;
    ++refinements;
    HIPCHK(hipMemsetAsync(xh, 0, NR * 16, st), "zero");
    int it = 0;
    if ((s = gmres_equilibrated(op, rhat, xh, (int)R, o, inner, 3 | (o.adjoint ? 4 : 0) | block, prec, &it, st,
                                work)))
      return s;
    iters += it;
    if ((e = pie::launch_scale_rows(xh, op->dDiagScale, N, (int)R, xh, st)) != hipSuccess) return hip_fail(e, "scale");
    std::vector<cx<double>> one(R, cx<double>{1.0, 0.0});
    HIPCHK(hipMemcpyAsync(dn, one.data(), R * 16, hipMemcpyHostToDevice, st), "one copy");
    if ((e = pie::launch_axpy_cols(X, xh, dn, N, (int)R, st)) != hipSuccess) return hip_fail(e, "axpy");
    HIPCHK(hipStreamSynchronize(st), "solve");
    if (k == o.refine - 1) {
      if ((s = solve_mvm(rop, X, zx, R, 3 | (o.adjoint ? 4 : 0) | block, st))) return s;
      if ((e = pie::launch_sub(b, zx, N, (int)R, rr, st)) != hipSuccess) return hip_fail(e, "sub");
      if ((s = dnorm(rr, rn))) return s;
      relmax = 0.0;
      for (int r = 0; r < R; ++r) relmax = std::max(relmax, bn[r] > 0 ? rn[r] / bn[r] : 0.0);
    }
  }
  if (info) {
    info->iterations = iters;
    info->refinements = refinements;
    info->rel_residual = relmax;
  }
  return relmax <= o.tol ? PIE_OK : PIE_WARN_NOT_CONVERGED;
}

extern "C" pie_status pie_solve(pie_op* op, pie_op* res_op, const void* b, void* x, int64_t R,
                                const pie_solve_opts* opts, pie_solve_info* info, void* stream) {
  return solve_core(op, res_op, b, x, R, opts, info, stream, 0);
}

// Workspace of pie_solve_noalloc: one array per GPU, loaded with the code
// object and kept until the process ends.  Host code uses its device address
// from hipGetSymbolAddress (per device), never the array's name.
static __device__ __align__(256) unsigned char scratch[PIE_SOLVE_NOALLOC_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on device dev, looked up once per device with
// that device current.
pie_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxScratchDevices) {
    pie::set_error("device index out of range for the solver scratch table");
    return PIE_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    HIPCHK(hipGetDevice(&cur), "hipGetDevice");
    if (cur != dev) HIPCHK(hipSetDevice(dev), "hipSetDevice");
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PIE_OK;
}
}  // namespace

extern "C" pie_status pie_solve_noalloc(pie_op* op, pie_op* res_op, const void* b, void* x, int64_t R,
                                        const pie_solve_opts* opts, pie_solve_info* info, void* stream) {
  if (!op) {
    pie::set_error("null operator");
    return PIE_ERR_ARG;
  }
  void* ws = nullptr;
  pie_status s = scratch_address(op->device, &ws);
  if (s) return s;
  return solve_core(op, res_op, b, x, R, opts, info, stream, 0, ws, PIE_SOLVE_NOALLOC_BYTES);
}

extern "C" pie_status pie_precond_apply(pie_op* op, const void* x, void* y, int64_t R, void* stream) {
  pie_status s = check_op_call(op, x, y, R);
  if (s) return s;
  if (!op->dPrec && (s = build_prec(op))) return s;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_block_prec(x, nullptr, op->dPrec, op->dPrecOff, op->dBoxPtr, op->dPerm,
                                   (int)op->tree->lev[op->L].nb, (int)R, y, st);
  if (e != hipSuccess) return hip_fail(e, "preconditioner");
  return PIE_OK;
}

extern "C" pie_status pie_charge(pie_op* op, int64_t R, const double* khat, const double* pol, const double* amp,
                                 int32_t gauge, const void* x, void* sigma, void* rho,
                                 const pie_solve_opts* opts, pie_solve_info* info, void* stream) {
  if (!op || !khat || !pol || !amp || !sigma || (rho && !x)) {
    pie::set_error("null argument (rho needs the PIE solution x)");
    return PIE_ERR_ARG;
  }
  if (R < 1 || R > op->max_rhs) {
    pie::set_error("R must be in [1, max_rhs]");
    return PIE_ERR_ARG;
  }
  if (opts && opts->adjoint) {
    pie::set_error("the charge solve has no adjoint");
    return PIE_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  const int N = op->N, E = op->ne, T = op->nt;
  const size_t NR = (size_t)N * R;
  cx<double>* buf = nullptr;
  HIPCHK(hipMalloc(&buf, 2 * NR * sizeof(cx<double>)), "charge workspace");
  std::unique_ptr<void, void (*)(void*)> guard(buf, [](void* p) { (void)hipFree(p); });
  cx<double>* b = buf;
  cx<double>* X = buf + NR;
  // right-hand side of Eq. (3) tested with the pulses, scaled by w^2 eps0 to
  // match the pulse-pulse block of Z: the plane-wave pulse rows are
  // -i w eps0 <P_q, Phi^inc>, times i w
  pie_status s = pie_rhs_planewave(op, R, khat, pol, amp, gauge, b, stream);
  if (s) return s;
  hipError_t e = pie::launch_pulse_rhs(b, E, N, (int)R, 0.0, op->omega, st);
  if (e != hipSuccess) return hip_fail(e, "charge rhs");
  pie_solve_opts o;
  pie_solve_opts_default(&o);
  if (opts) {
    if (opts->version == 1) {
      std::memcpy(&o, opts, offsetof(pie_solve_opts, precond));
    } else if (opts->version == 2) {
      o = *opts;
    } else {
      pie::set_error("pie_solve_opts.version must be 1 or 2");
      return PIE_ERR_ARG;
    }
  }
  o.version = 2;
  o.use_x0 = 0;
  o.precond = 0;  // the self blocks are those of the whole operator
  s = solve_core(op, nullptr, b, X, R, &o, info, stream, SOLVE_PULSE_BLOCK);
  if (s != PIE_OK && s != PIE_WARN_NOT_CONVERGED) return s;
  // sigma = pulse rows of the block solution; rho = i w eps0 (n.A) - eps0 sigma
  HIPCHK(hipMemcpyAsync(sigma, X + (size_t)E * R, (size_t)T * R * sizeof(cx<double>), hipMemcpyDeviceToDevice, st),
         "sigma copy");
  if (rho) {
    e = pie::launch_charge_rho((const cx<double>*)x + (size_t)E * R, (const cx<double>*)sigma, (int64_t)T * R,
                               op->omega * pie::kEps0, pie::kEps0, rho, st);
    if (e != hipSuccess) return hip_fail(e, "rho");
  }
  HIPCHK(hipStreamSynchronize(st), "charge");
  return s;
}
