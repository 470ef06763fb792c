// Far field of the MLFMA (Section 3): radiation patterns and aggregation,
// diagonal translation with the scaled plane waves of Eq. (4) and the
// modified translation function of Eq. (5), disaggregation and reception.
//
// Pattern layout (outgoing S and incoming G of every level), box-major:
//   P[(box * Q + q) * 5R + c * R + r],  c in {Jx, Jy, Jz, sigma, u},
// u = div J + w^2 eps0 sigma, R = the RHS columns of the launch.  A box's
// Q x 5R values are contiguous, so the translation's gather of one source
// box by the Q sample lanes of a workgroup is a single contiguous run.
#include <algorithm>

#include "device.h"
#include "kernels.h"

namespace pie {

// ---------------------------------------------------------------------------
// Finest-level aggregation.  Every (box, triangle) incidence contributes
// seven quadrature points; per point the source density
//   W_i * (J(r_i), sigma, div J + w^2 eps0 sigma),  J = sum x_n s_n (r_i - p_n)
// is formed from x (independent loads of the incidence tables, then of x),
// then for every sample q
//   S(q) += density * exp(-i kappa khat_q . (r_i - C_box)).
// Workgroup = one finest box; stage 1 threads over points, stage 2 over
// (q, point slice), stage 3 adds the slices in a fixed order.
// ---------------------------------------------------------------------------
template <typename TF, int RC, int NT>
__global__ void __launch_bounds__(256) k_aggregate(DevInc I, int nbox, const cx<double>* __restrict__ x, int ldx,
                                                   const TF* __restrict__ khat, int Q, TF kappa, double w2e,
                                                   int conjx, int nsplit, cx<TF>* __restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_box(blockIdx.x, nbox);
  if (b < 0) return;
  const int j0 = I.ptr[b], j1 = I.ptr[b + 1];
  const int npt = 7 * (j1 - j0);
  constexpr int ncol = 5 * RC;
  cx<TF>* dens = (cx<TF>*)smem;                              // [npt][5][RC]
  cx<TF>* part = dens + (size_t)npt * ncol;                  // [nsplit][Q][5][RC]
  TF* poff = (TF*)(part + (size_t)nsplit * Q * ncol);        // [npt][4]
  for (int p = threadIdx.x; p < npt; p += blockDim.x) {
    const int j = j0 + p / 7;
    const double* pw = I.pw + 4 * ((size_t)7 * j0 + p);
    const double o[3] = {pw[0], pw[1], pw[2]}, w = pw[3];
    int xc[4];
    double sv[3], dv[3], pv[3][3];
#pragma unroll
    for (int k = 0; k < 4; ++k) xc[k] = I.xc[4 * (size_t)j + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sv[k] = I.rs[3 * (size_t)j + k];
      dv[k] = I.rd[3 * (size_t)j + k];
#pragma unroll
      for (int c = 0; c < 3; ++c) pv[k][c] = I.pv[9 * (size_t)j + 3 * k + c];
    }
    poff[4 * p + 0] = (TF)o[0];
    poff[4 * p + 1] = (TF)o[1];
    poff[4 * p + 2] = (TF)o[2];
    poff[4 * p + 3] = (TF)0;
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      cx<double> xv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xv[k] = xc[k] >= 0 ? x[(size_t)xc[k] * ldx + r] : mk(0.0, 0.0);
        if (conjx) xv[k].im = -xv[k].im;
      }
      cx<double> J[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
      cx<double> D = mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) J[c] = J[c] + (sv[k] * (o[c] - pv[k][c])) * xv[k];
        D = D + dv[k] * xv[k];
      }
      const cx<double> sg = xv[3];
      cx<TF>* dp = dens + (size_t)p * ncol;
#pragma unroll
      for (int c = 0; c < 3; ++c) dp[c * RC + r] = mk((TF)(w * J[c].re), (TF)(w * J[c].im));
      dp[3 * RC + r] = mk((TF)(w * sg.re), (TF)(w * sg.im));
      const cx<double> uu = D + w2e * sg;
      dp[4 * RC + r] = mk((TF)(w * uu.re), (TF)(w * uu.im));
    }
  }
  __syncthreads();
  if (threadIdx.x < nsplit * Q) {
    const int q = threadIdx.x % Q, part_id = threadIdx.x / Q;
    const TF kx = kappa * khat[3 * q], ky = kappa * khat[3 * q + 1], kz = kappa * khat[3 * q + 2];
    cx<TF> acc[ncol];
#pragma unroll
    for (int c = 0; c < ncol; ++c) acc[c] = mk<TF>(0, 0);
    // two points per step (same per-accumulator order as one at a time)
    int p = part_id;
    for (; p + nsplit < npt; p += 2 * nsplit) {
      const TF* o0 = poff + 4 * p;
      const TF* o1 = poff + 4 * (p + nsplit);
      cx<TF> d0[ncol], d1[ncol];
#pragma unroll
      for (int c = 0; c < ncol; ++c) {
        d0[c] = dens[(size_t)p * ncol + c];
        d1[c] = dens[(size_t)(p + nsplit) * ncol + c];
      }
      const TF th0 = kx * o0[0] + ky * o0[1] + kz * o0[2];
      const TF th1 = kx * o1[0] + ky * o1[1] + kz * o1[2];
      TF s0, c0, s1, c1;
      phase<TF, NT>(th0, &s0, &c0);
      phase<TF, NT>(th1, &s1, &c1);
      const cx<TF> e0 = mk(c0, -s0), e1 = mk(c1, -s1);
#pragma unroll
      for (int c = 0; c < ncol; ++c) {
        cfma(acc[c], d0[c], e0);
        cfma(acc[c], d1[c], e1);
      }
    }
    if (p < npt) {
      const TF* o0 = poff + 4 * p;
      const TF th0 = kx * o0[0] + ky * o0[1] + kz * o0[2];
      TF s0, c0;
      phase<TF, NT>(th0, &s0, &c0);
      const cx<TF> e0 = mk(c0, -s0);
#pragma unroll
      for (int c = 0; c < ncol; ++c) cfma(acc[c], dens[(size_t)p * ncol + c], e0);
    }
    cx<TF>* pp = part + ((size_t)part_id * Q + q) * ncol;
#pragma unroll
    for (int c = 0; c < ncol; ++c) pp[c] = acc[c];
  }
  __syncthreads();
  // fixed-order combination of the partial sums; dens is [comp][RC] = col order
  for (int e = threadIdx.x; e < Q * ncol; e += blockDim.x) {
    const int q = e / ncol, c = e - q * ncol;
    cx<TF> v = part[(size_t)q * ncol + c];
    for (int h = 1; h < nsplit; ++h) v = v + part[((size_t)h * Q + q) * ncol + c];
    S[((size_t)b * Q + q) * ncol + c] = v;
  }
}

// ---------------------------------------------------------------------------
// Inter-level shifts as small GEMMs.  A workgroup owns a group of at most
// SHIFT_GROUP boxes and a tile of SQT sample rows.  Its filter rows are
// staged once in LDS; a lane owns one (box, column) pair and accumulates its
// SQT outputs over a slice of the Q input samples (nsl slices, one per
// wavefront group, combined through LDS in a fixed order), so every loaded
// pattern value feeds SQT fused multiply-adds and each lane walks a short
// run of independent loads.  The filter tables carry SQT zero entries of
// padding so that the last, partial row tile reads in bounds.
//
// Child -> parent:  S_p(q) = sum_c exp(-i kappa_p khat_q.(C_c - C_p))
//                                  * sum_q' F[q][q'] S_c(q')   (Ft = F^T)
// The group is a run of parents whose children (contiguous in Morton order)
// number at most SHIFT_GROUP; the phased child rows go to LDS and each
// parent sums them in Morton order (fixed order, no atomics).
// ---------------------------------------------------------------------------
template <typename TF>
__device__ __forceinline__ void shift_tile(const TF* __restrict__ Fsrc, TF* Fs, int Q, int q0) {
  for (int e = threadIdx.x; e < Q * SQT; e += blockDim.x) {
    const int qq = e / SQT, i = e - qq * SQT;
    Fs[e] = Fsrc[(size_t)qq * Q + q0 + i];
  }
}

// acc[i] = sum_{q' in slice} Fs[q'][i] * v(q'), v(q') = load(q'); the
// loads of eight samples are issued together before their arithmetic.
template <typename TF>
__device__ __forceinline__ void shift_fma(const TF* f, const cx<TF>& v, cx<TF>* acc) {
#pragma unroll
  for (int i = 0; i < SQT; ++i) {
    acc[i].re = fma(f[i], v.re, acc[i].re);
    acc[i].im = fma(f[i], v.im, acc[i].im);
  }
}

template <typename TF, typename LD>
__device__ __forceinline__ void shift_mac(const TF* Fs, int qa, int qb, LD load, cx<TF>* acc) {
  constexpr int U = 8;
  int qq = qa;
  for (; qq + U <= qb; qq += U) {
    cx<TF> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load(qq + u);
    __builtin_amdgcn_sched_barrier(0);  // keep the eight loads in flight together
#pragma unroll
    for (int u = 0; u < U; ++u) shift_fma(Fs + (qq + u) * SQT, v[u], acc);
  }
  for (; qq < qb; ++qq) shift_fma(Fs + qq * SQT, load(qq), acc);
}

// Work item of a shift launch: blockIdx -> (group, row tile, RHS column) with
// the groups of an XCD contiguous (workgroups go round-robin over 8 XCDs).
struct ShiftItem {
  int g, q0, r;
};
__device__ __forceinline__ bool shift_item(int ngroup, int ntile, int R, ShiftItem& it) {
  const int per = (ngroup + 7) >> 3, w = blockIdx.x, x = w & 7, j = w >> 3;
  const int sub = ntile * R, gl = j / sub, rem = j - gl * sub;
  it.g = x * per + gl;
  it.q0 = (rem / R) * SQT;
  it.r = rem - (rem / R) * R;
  return gl < per && it.g < ngroup;
}

// One slice-lane layout for both shifts: 64 lanes = SHIFT_GROUP boxes x 5
// components (of one RHS column), SHIFT_SLICES slices of the Q sum.
constexpr int SHIFT_LANES = 64;
constexpr int SHIFT_SLICES = 4;

template <typename TF>
__global__ void __launch_bounds__(256) k_shift_up(DevLevel Lp, DevLevel Lc,
                                                  const cx<TF>* __restrict__ Sc, cx<TF>* __restrict__ Sp,
                                                  const TF* __restrict__ Ft, const cx<TF>* __restrict__ ph,
                                                  int Q, int R, int ntile) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<TF>* part = (cx<TF>*)smem;                               // [slice][lane][SQT]
  TF* Fs = (TF*)(part + (size_t)SHIFT_SLICES * SHIFT_LANES * SQT);  // [Q][SQT]
  ShiftItem it;
  if (!shift_item(Lp.nug, ntile, R, it)) return;
  const int q0 = it.q0, r = it.r;
  const int nq = min(SQT, Q - q0);
  shift_tile(Ft, Fs, Q, q0);
  __syncthreads();
  const int p0 = Lp.ug_ptr[it.g], p1 = Lp.ug_ptr[it.g + 1];
  const int c0 = Lp.child_ptr[p0], c1 = Lp.child_ptr[p1];
  const int t = threadIdx.x, sl = t / SHIFT_LANES, lane = t - sl * SHIFT_LANES;
  const int ci = lane / 5, k = lane - ci * 5;
  const int c = c0 + ci;
  const bool act = ci < SHIFT_GROUP && c < c1;
  const int qs = (Q + SHIFT_SLICES - 1) / SHIFT_SLICES, qa = sl * qs, qb = min(Q, qa + qs);
  cx<TF> acc[SQT];
#pragma unroll
  for (int i = 0; i < SQT; ++i) acc[i] = mk<TF>(0, 0);
  if (act) {
    const int ncol = 5 * R;
    const cx<TF>* s = Sc + (size_t)c * Q * ncol + k * R + r;
    shift_mac(Fs, qa, qb, [&](int qq) { return s[(size_t)qq * ncol]; }, acc);
  }
  if (sl > 0) {
#pragma unroll
    for (int i = 0; i < SQT; ++i) part[(size_t)t * SQT + i] = acc[i];
  }
  __syncthreads();
  if (sl == 0 && act) {
    const cx<TF>* pc = ph + (size_t)Lc.octant[c] * Q + q0;
    for (int h = 1; h < SHIFT_SLICES; ++h)
#pragma unroll
      for (int i = 0; i < SQT; ++i) acc[i] = acc[i] + part[((size_t)h * SHIFT_LANES + lane) * SQT + i];
#pragma unroll
    for (int i = 0; i < SQT; ++i)
      if (i < nq) part[(size_t)lane * SQT + i] = pc[i] * acc[i];
  }
  __syncthreads();
  const int np = p1 - p0, m = np * nq * 5;
  for (int e = t; e < m; e += blockDim.x) {
    const int pl = e / (nq * 5), rem = e - pl * nq * 5;
    const int i = rem / 5, kk = rem - i * 5;
    const int p = p0 + pl;
    cx<TF> v = mk<TF>(0, 0);
    for (int ch = Lp.child_ptr[p]; ch < Lp.child_ptr[p + 1]; ++ch) v = v + part[((ch - c0) * 5 + kk) * SQT + i];
    Sp[((size_t)p * Q + q0 + i) * 5 * R + kk * R + r] = v;
  }
}

// Parent -> child:  G_c(q) += sum_q' F[q'][q] exp(+i kappa_p khat_q'.(C_c - C_p)) G_p(q')
// (the transpose of the upward filter, conjugate phase).  The group is a run
// of SHIFT_GROUP consecutive boxes of the child level.
template <typename TF>
__global__ void __launch_bounds__(256) k_shift_down(DevLevel Lc, const cx<TF>* __restrict__ Gp,
                                                    cx<TF>* __restrict__ Gc, const TF* __restrict__ F,
                                                    const cx<TF>* __restrict__ ph, int Q, int R, int ntile) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<TF>* part = (cx<TF>*)smem;                               // [slice][lane][SQT]
  TF* Fs = (TF*)(part + (size_t)SHIFT_SLICES * SHIFT_LANES * SQT);  // [Q][SQT]
  const int ng = (Lc.nb + SHIFT_GROUP - 1) / SHIFT_GROUP;
  ShiftItem it;
  if (!shift_item(ng, ntile, R, it)) return;
  const int q0 = it.q0, r = it.r;
  const int nq = min(SQT, Q - q0);
  shift_tile(F, Fs, Q, q0);
  __syncthreads();
  const int t = threadIdx.x, sl = t / SHIFT_LANES, lane = t - sl * SHIFT_LANES;
  const int ci = lane / 5, k = lane - ci * 5;
  const int c = it.g * SHIFT_GROUP + ci;
  const bool act = ci < SHIFT_GROUP && c < Lc.nb;
  const int qs = (Q + SHIFT_SLICES - 1) / SHIFT_SLICES, qa = sl * qs, qb = min(Q, qa + qs);
  cx<TF> acc[SQT];
#pragma unroll
  for (int i = 0; i < SQT; ++i) acc[i] = mk<TF>(0, 0);
  if (act) {
    const int ncol = 5 * R;
    const cx<TF>* gp = Gp + (size_t)Lc.parent[c] * Q * ncol + k * R + r;
    const cx<TF>* pc = ph + (size_t)Lc.octant[c] * Q;
    shift_mac(Fs, qa, qb, [&](int qq) { return conj(pc[qq]) * gp[(size_t)qq * ncol]; }, acc);
  }
  if (sl > 0) {
#pragma unroll
    for (int i = 0; i < SQT; ++i) part[(size_t)t * SQT + i] = acc[i];
  }
  __syncthreads();
  if (sl == 0 && act) {
    for (int h = 1; h < SHIFT_SLICES; ++h)
#pragma unroll
      for (int i = 0; i < SQT; ++i) acc[i] = acc[i] + part[((size_t)h * SHIFT_LANES + lane) * SQT + i];
    const int ncol = 5 * R;
    cx<TF>* o = Gc + ((size_t)c * Q + q0) * ncol + k * R + r;
#pragma unroll
    for (int i = 0; i < SQT; ++i)
      if (i < nq) o[(size_t)i * ncol] = o[(size_t)i * ncol] + acc[i];
  }
}

// ---------------------------------------------------------------------------
// Translation over the interaction list at one level:
//   G_b(q) = sum_{b' in IL(b)} T_{off(b,b')}(q) S_b'(q)
// a gather (no atomics).  One workgroup per (box, RHS column); the list is
// staged in LDS, thread (g, q) takes the entries g (mod nsplit) for all five
// components with four entries' loads in flight, and the nsplit partial
// sums are added in a fixed order through LDS.  nsplit depends on Q only,
// so every RHS column is summed in the same order.
// ---------------------------------------------------------------------------
template <typename TF>
__global__ void __launch_bounds__(512) k_translate(DevLevel Lv, const cx<TF>* __restrict__ S,
                                                   const cx<TF>* __restrict__ T, cx<TF>* __restrict__ Gout,
                                                   int Q, int R, int nsplit) {
  extern __shared__ __align__(16) unsigned char smem[];
  int32_t* ils = (int32_t*)smem;                 // [IL_MAX + 3]
  int32_t* ilo = ils + (IL_MAX + 3);             // [IL_MAX + 3]
  cx<TF>* part = (cx<TF>*)(ilo + (IL_MAX + 3));  // [nsplit - 1][width][5]
  const int b = xcd_box(blockIdx.x, Lv.nb);
  if (b < 0) return;
  const int r = blockIdx.y;
  const int ncol = 5 * R;
  const int n = Q * ncol;
  const int i0 = Lv.il_ptr[b], nil = Lv.il_ptr[b + 1] - i0;
  for (int e = threadIdx.x; e < nil; e += blockDim.x) {
    ils[e] = Lv.il_src[i0 + e];
    ilo[e] = Lv.il_off[i0 + e];
  }
  __syncthreads();
  const int width = blockDim.x / nsplit;
  const int gsp = threadIdx.x / width;
  constexpr int U = 4;
  for (int base = 0; base < Q; base += width) {
    const int q = base + threadIdx.x % width;
    const bool act = q < Q;
    cx<TF> acc[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k] = mk<TF>(0, 0);
    if (act) {
      const cx<TF>* Sq = S + (size_t)q * ncol + r;
      for (int kk = gsp; kk < nil; kk += U * nsplit) {
        cx<TF> tv[U], sv[U][5];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = kk + u * nsplit;
          const bool ok = e < nil;
          tv[u] = ok ? T[(size_t)ilo[e] * Q + q] : mk<TF>(0, 0);
          const cx<TF>* sp = Sq + (size_t)(ok ? ils[e] : 0) * n;
#pragma unroll
          for (int k = 0; k < 5; ++k) sv[u][k] = sp[k * R];
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the entries' loads in flight together
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int k = 0; k < 5; ++k) cfma(acc[k], tv[u], sv[u][k]);
      }
      if (gsp > 0) {
        cx<TF>* pp = part + ((size_t)(gsp - 1) * width + (q - base)) * 5;
#pragma unroll
        for (int k = 0; k < 5; ++k) pp[k] = acc[k];
      }
    }
    __syncthreads();
    if (act && gsp == 0) {
      for (int h = 1; h < nsplit; ++h) {
        const cx<TF>* pp = part + ((size_t)(h - 1) * width + (q - base)) * 5;
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[k] = acc[k] + pp[k];
      }
      cx<TF>* o = Gout + (size_t)b * n + (size_t)q * ncol + r;
#pragma unroll
      for (int k = 0; k < 5; ++k) o[k * R] = acc[k];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Reception at the finest level and join with the near-field partial sums.
// Per quadrature point the incoming field
//   fld(r_i) = W_i sum_q exp(+i kappa khat_q.(r_i - C_box)) G(q)
// is formed; then every unknown of the box takes its testing integral:
//   RWG:   y += mu0 s (r_i - p).fld_J + d fld_sigma   (both halves)
//   pulse: y += fld_u,
// adds its near-field partial sums in a fixed order (slot lists staged in
// LDS), and is written to the canonical position (conjugated for the
// adjoint).  Point offsets are kept in FP64 for the testing integrals.
// ---------------------------------------------------------------------------
template <typename TF, typename TN, int RC, int NT>
__global__ void __launch_bounds__(256) k_receive(DevInc I, DevBasis B, DevNear NB, int nbox,
                                                 const cx<TF>* __restrict__ Gin, const TF* __restrict__ khat,
                                                 int Q, TF kappa, const cx<TN>* __restrict__ part, int flags,
                                                 cx<double>* __restrict__ y, int ldy) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_box(blockIdx.x, nbox);
  if (b < 0) return;
  const int j0 = I.ptr[b], j1 = I.ptr[b + 1];
  const int npt = 7 * (j1 - j0);
  constexpr int ncol = 5 * RC;
  const bool do_far = flags & 2, do_near = flags & 1, conj_out = flags & 4;
  double* po = (double*)smem;                              // [npt][4] r_i - C, W_i
  cx<TF>* fld = (cx<TF>*)(po + 4 * (size_t)npt);            // [npt][5][RC]
  cx<TF>* Gs = fld + (size_t)npt * ncol;                   // [Q][5][RC]
  TF* kh = (TF*)(Gs + (size_t)Q * ncol);                   // [Q][4] kappa * khat
  int32_t* slots = (int32_t*)(kh + 4 * Q);                 // near-field partial-sum slots
  const double mu0 = 4.0e-7 * 3.14159265358979323846;
  const int nrow = do_near ? NB.row_ptr[b + 1] - NB.row_ptr[b] : 0;
  const int nslot = do_near ? nrow + NB.col_ptr[b + 1] - NB.col_ptr[b] : 0;
  for (int e = threadIdx.x; e < nslot; e += blockDim.x)
    slots[e] = e < nrow ? NB.prow[NB.row_ptr[b] + e] : NB.pcol[NB.col_blk[NB.col_ptr[b] + e - nrow]];
  if (do_far) {
    const cx<TF>* g = Gin + (size_t)b * Q * ncol;
    for (int e = threadIdx.x; e < Q * ncol; e += blockDim.x) Gs[e] = g[e];
    for (int q = threadIdx.x; q < Q; q += blockDim.x) {
      kh[4 * q + 0] = kappa * khat[3 * q];
      kh[4 * q + 1] = kappa * khat[3 * q + 1];
      kh[4 * q + 2] = kappa * khat[3 * q + 2];
      kh[4 * q + 3] = 0;
    }
    const double* pw = I.pw + 28 * (size_t)j0;
    for (int e = threadIdx.x; e < 4 * npt; e += blockDim.x) po[e] = pw[e];
  }
  __syncthreads();
  if (do_far) {
    for (int p = threadIdx.x; p < npt; p += blockDim.x) {
      cx<TF> acc[ncol];
#pragma unroll
      for (int c = 0; c < ncol; ++c) acc[c] = mk<TF>(0, 0);
      const TF ox = (TF)po[4 * p], oy = (TF)po[4 * p + 1], oz = (TF)po[4 * p + 2];
#pragma unroll 2
      for (int q = 0; q < Q; ++q) {
        const TF* k4 = kh + 4 * q;
        cx<TF> gq[ncol];
#pragma unroll
        for (int c = 0; c < ncol; ++c) gq[c] = Gs[(size_t)q * ncol + c];
        const TF th = k4[0] * ox + k4[1] * oy + k4[2] * oz;
        TF sn, cs;
        phase<TF, NT>(th, &sn, &cs);
        const cx<TF> e = mk(cs, sn);
#pragma unroll
        for (int c = 0; c < ncol; ++c) cfma(acc[c], e, gq[c]);
      }
      const TF w = (TF)po[4 * p + 3];
      cx<TF>* fp = fld + (size_t)p * ncol;
#pragma unroll
      for (int c = 0; c < ncol; ++c) fp[c] = w * acc[c];
    }
    __syncthreads();
  }
  const int u0 = NB.box_ptr[b], nu = NB.box_ptr[b + 1] - u0;
  for (int e = threadIdx.x; e < nu * RC; e += blockDim.x) {
    const int ul = e / RC, r = e - ul * RC;
    const int u = u0 + ul;
    const int cu = B.perm[u];
    cx<double> val = mk(0.0, 0.0);
    if (do_far) {
      if (cu < B.ne) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int jl = I.uj[2 * u + h] - j0;
          const double s = I.us[2 * u + h], d = I.ud[2 * u + h];
          const double pv[3] = {I.upv[6 * (size_t)u + 3 * h], I.upv[6 * (size_t)u + 3 * h + 1],
                                I.upv[6 * (size_t)u + 3 * h + 2]};
#pragma unroll
          for (int i = 0; i < 7; ++i) {
            const double* o = po + 4 * (7 * jl + i);
            const cx<TF>* f = fld + (size_t)(7 * jl + i) * ncol;
            cx<double> a = mk(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const double dd = mu0 * s * (o[c] - pv[c]);
              a.re += dd * (double)f[c * RC + r].re;
              a.im += dd * (double)f[c * RC + r].im;
            }
            a.re += d * (double)f[3 * RC + r].re;
            a.im += d * (double)f[3 * RC + r].im;
            val = val + a;
          }
        }
      } else {
        const int jl = I.uj[2 * u] - j0;
        const cx<TF>* fp = fld + (size_t)jl * 7 * ncol;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
          val.re += (double)fp[(size_t)i * ncol + 4 * RC + r].re;
          val.im += (double)fp[(size_t)i * ncol + 4 * RC + r].im;
        }
      }
    }
    if (do_near) {
      int k = 0;
      for (; k + 4 <= nslot; k += 4) {
        cx<TN> v[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = part[((size_t)slots[k + t] + ul) * RC + r];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          val.re += (double)v[t].re;
          val.im += (double)v[t].im;
        }
      }
      for (; k < nslot; ++k) {
        const cx<TN> v = part[((size_t)slots[k] + ul) * RC + r];
        val.re += (double)v.re;
        val.im += (double)v.im;
      }
    }
    if (conj_out) val.im = -val.im;
    y[(size_t)cu * ldy + r] = val;
  }
}

// Canonical FP64 x -> box-order x in near-field precision (conjugated for
// the adjoint).
template <typename TN>
__global__ void k_permute_in(const cx<double>* __restrict__ x, int ldx, const int32_t* __restrict__ perm,
                             int N, int R, int conjx, cx<TN>* __restrict__ xb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * R) return;
  const int u = (int)(e / R), r = (int)(e - (int64_t)u * R);
  cx<double> v = x[(size_t)perm[u] * ldx + r];
  if (conjx) v.im = -v.im;
  xb[e] = mk((TN)v.re, (TN)v.im);
}

// ------------------------------------------------------------- launchers --
size_t aggregate_smem(int maxpt, int Q, int nsplit, int RC, int tf_bytes) {
  return (size_t)maxpt * 5 * RC * 2 * tf_bytes + (size_t)nsplit * Q * 5 * RC * 2 * tf_bytes +
         (size_t)maxpt * 4 * tf_bytes + 16;
}
size_t receive_smem(int maxpt, int Q, int maxjoin, int RC, int tf_bytes) {
  return (size_t)maxpt * 4 * 8 + (size_t)maxpt * 5 * RC * 2 * tf_bytes + (size_t)Q * 5 * RC * 2 * tf_bytes +
         (size_t)Q * 4 * tf_bytes + (size_t)maxjoin * 4 + 16;
}

template <typename TF, int RC, int NT>
static void agg_launch(const DevInc& I, int nb, int maxpt, const void* x, int ldx, const void* khat, int Q,
                       double kappa, double w2e, int conjx, int nsplit, void* S, hipStream_t st) {
  size_t sm = aggregate_smem(maxpt, Q, nsplit, RC, sizeof(TF));
  hipLaunchKernelGGL((k_aggregate<TF, RC, NT>), dim3(xcd_grid(nb)), dim3(256), sm, st, I, nb, (const cx<double>*)x,
                     ldx, (const TF*)khat, Q, (TF)kappa, w2e, conjx, nsplit, (cx<TF>*)S);
}

template <typename TF>
hipError_t launch_aggregate(const DevInc& I, int nb, int maxpt, const void* x, int ldx, int R, const void* khat,
                            int Q, double kappa, double w2e, int conjx, int nsplit, int phase_mode, void* S,
                            hipStream_t st) {
  constexpr int NS = sizeof(TF) == 8 ? 5 : 4, NL = sizeof(TF) == 8 ? 9 : 6;
  if (R != 1 && R != 2 && R != 4) return hipErrorInvalidValue;
#define AGG(RC_, NT_) agg_launch<TF, RC_, NT_>(I, nb, maxpt, x, ldx, khat, Q, kappa, w2e, conjx, nsplit, S, st)
  if (phase_mode == 1) {
    if (R == 1) AGG(1, NS); else if (R == 2) AGG(2, NS); else AGG(4, NS);
  } else if (phase_mode == 2) {
    if (R == 1) AGG(1, NL); else if (R == 2) AGG(2, NL); else AGG(4, NL);
  } else {
    if (R == 1) AGG(1, 0); else if (R == 2) AGG(2, 0); else AGG(4, 0);
  }
#undef AGG
  return hipGetLastError();
}

size_t shift_smem(int Q, int tf_bytes) {
  return (size_t)SHIFT_SLICES * SHIFT_LANES * SQT * 2 * tf_bytes + (size_t)Q * SQT * tf_bytes;
}

template <typename TF>
hipError_t launch_shift_up(const DevLevel& Lp, const DevLevel& Lc, const void* Sc, void* Sp, const void* Ft,
                           const void* ph, int Q, int R, hipStream_t st) {
  static_assert(SHIFT_GROUP * 5 <= SHIFT_LANES, "shift group exceeds its lanes");
  const int ntile = (Q + SQT - 1) / SQT;
  const unsigned grid = 8u * (unsigned)(((Lp.nug + 7) / 8) * ntile * R);
  hipLaunchKernelGGL(k_shift_up<TF>, dim3(grid), dim3(SHIFT_SLICES * SHIFT_LANES), shift_smem(Q, sizeof(TF)), st,
                     Lp, Lc, (const cx<TF>*)Sc, (cx<TF>*)Sp, (const TF*)Ft, (const cx<TF>*)ph, Q, R, ntile);
  return hipGetLastError();
}

template <typename TF>
hipError_t launch_shift_down(const DevLevel& Lc, const void* Gp, void* Gc, const void* F, const void* ph, int Q,
                             int R, hipStream_t st) {
  const int ntile = (Q + SQT - 1) / SQT;
  const int ng = (Lc.nb + SHIFT_GROUP - 1) / SHIFT_GROUP;
  const unsigned grid = 8u * (unsigned)(((ng + 7) / 8) * ntile * R);
  hipLaunchKernelGGL(k_shift_down<TF>, dim3(grid), dim3(SHIFT_SLICES * SHIFT_LANES), shift_smem(Q, sizeof(TF)),
                     st, Lc, (const cx<TF>*)Gp, (cx<TF>*)Gc, (const TF*)F, (const cx<TF>*)ph, Q, R, ntile);
  return hipGetLastError();
}

// Interaction-list split: Q lanes rounded to wavefronts (at most 256 per
// pass) times nsplit list slices in a block of at most 512 threads.
int translate_width(int Q) { return std::min(256, 64 * ((Q + 63) / 64)); }
int translate_split(int Q) { return std::min(8, 512 / translate_width(Q)); }

template <typename TF>
hipError_t launch_translate(const DevLevel& Lv, const void* S, const void* T, void* Gout, int Q, int R,
                            hipStream_t st) {
  const int width = translate_width(Q), ns = translate_split(Q);
  const size_t sm = 2 * (IL_MAX + 3) * sizeof(int32_t) + (size_t)(ns - 1) * width * 5 * 2 * sizeof(TF) + 16;
  hipLaunchKernelGGL(k_translate<TF>, dim3(xcd_grid(Lv.nb), R), dim3(width * ns), sm, st, Lv, (const cx<TF>*)S,
                     (const cx<TF>*)T, (cx<TF>*)Gout, Q, R, ns);
  return hipGetLastError();
}

template <typename TF, typename TN, int RC, int NT>
static void rec_launch(const DevInc& I, const DevBasis& B, const DevNear& NB, int nb, int maxpt, int maxjoin,
                       const void* Gin, const void* khat, int Q, double kappa, const void* part, int flags, void* y,
                       int ldy, hipStream_t st) {
  size_t sm = receive_smem(maxpt, Q, maxjoin, RC, sizeof(TF));
  hipLaunchKernelGGL((k_receive<TF, TN, RC, NT>), dim3(xcd_grid(nb)), dim3(256), sm, st, I, B, NB, nb,
                     (const cx<TF>*)Gin, (const TF*)khat, Q, (TF)kappa, (const cx<TN>*)part, flags,
                     (cx<double>*)y, ldy);
}

template <typename TF, typename TN>
hipError_t launch_receive(const DevInc& I, const DevBasis& B, const DevNear& NB, int nb, int maxpt, int maxjoin,
                          const void* Gin, const void* khat, int Q, double kappa, const void* part, int R,
                          int flags, int phase_mode, void* y, int ldy, hipStream_t st) {
  constexpr int NS = sizeof(TF) == 8 ? 5 : 4, NL = sizeof(TF) == 8 ? 9 : 6;
  if (R != 1 && R != 2 && R != 4) return hipErrorInvalidValue;
#define REC(RC_, NT_) \
  rec_launch<TF, TN, RC_, NT_>(I, B, NB, nb, maxpt, maxjoin, Gin, khat, Q, kappa, part, flags, y, ldy, st)
  if (phase_mode == 1) {
    if (R == 1) REC(1, NS); else if (R == 2) REC(2, NS); else REC(4, NS);
  } else if (phase_mode == 2) {
    if (R == 1) REC(1, NL); else if (R == 2) REC(2, NL); else REC(4, NL);
  } else {
    if (R == 1) REC(1, 0); else if (R == 2) REC(2, 0); else REC(4, 0);
  }
#undef REC
  return hipGetLastError();
}

template <typename TN>
hipError_t launch_permute_in(const void* x, int ldx, const int32_t* perm, int N, int R, int conjx, void* xb,
                             hipStream_t st) {
  int64_t n = (int64_t)N * R;
  hipLaunchKernelGGL(k_permute_in<TN>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const cx<double>*)x, ldx, perm, N, R, conjx, (cx<TN>*)xb);
  return hipGetLastError();
}

#define INST_F(TF)                                                                                            \
  template hipError_t launch_aggregate<TF>(const DevInc&, int, int, const void*, int, int, const void*, int,    \
                                           double, double, int, int, int, void*, hipStream_t);              \
  template hipError_t launch_shift_up<TF>(const DevLevel&, const DevLevel&, const void*, void*, const void*,  \
                                          const void*, int, int, hipStream_t);                               \
  template hipError_t launch_shift_down<TF>(const DevLevel&, const void*, void*, const void*, const void*,   \
                                            int, int, hipStream_t);                                          \
  template hipError_t launch_translate<TF>(const DevLevel&, const void*, const void*, void*, int, int,       \
                                           hipStream_t);                                                     \
  template hipError_t launch_permute_in<TF>(const void*, int, const int32_t*, int, int, int, void*,           \
                                            hipStream_t);
INST_F(float)
INST_F(double)
template hipError_t launch_receive<float, float>(const DevInc&, const DevBasis&, const DevNear&, int, int, int, const void*, const void*, int, double, const void*, int, int, int, void*, int, hipStream_t);
template hipError_t launch_receive<double, float>(const DevInc&, const DevBasis&, const DevNear&, int, int, int, const void*, const void*, int, double, const void*, int, int, int, void*, int, hipStream_t);
template hipError_t launch_receive<float, double>(const DevInc&, const DevBasis&, const DevNear&, int, int, int, const void*, const void*, int, double, const void*, int, int, int, void*, int, hipStream_t);
template hipError_t launch_receive<double, double>(const DevInc&, const DevBasis&, const DevNear&, int, int, int, const void*, const void*, int, double, const void*, int, int, int, void*, int, hipStream_t);

}  // namespace pie
