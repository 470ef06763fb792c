// Far field of the MLFMA (Section 3): radiation patterns and aggregation,
// diagonal translation with the scaled plane waves of Eq. (4) and the
// modified translation function of Eq. (5), disaggregation and reception.
//
// Pattern layout: S[box][q][col], col = c * R + r, c in {Jx, Jy, Jz, sigma,
// u}, u = div J + w^2 eps0 sigma; sample-major within a box so that a
// workgroup reads one box's Q x 5R values contiguously.
#include "device.h"
#include "kernels.h"

namespace pie {

// ---------------------------------------------------------------------------
// Finest-level aggregation.  Every (box, triangle) incidence contributes
// seven quadrature points; per point the source density
//   W_i * (J(r_i), sigma, div J + w^2 eps0 sigma),  J = sum x_n s_n (r_i - p_n)
// is formed from x, then for every sample q
//   S(q) += density * exp(-i kappa khat_q . (r_i - C_box)).
// Workgroup = one finest box; stage 1 threads over points, stage 2 over q.
// ---------------------------------------------------------------------------
template <typename TF, int RC, int NT>
__global__ void __launch_bounds__(256) k_aggregate(DevGeo G, DevInc I, DevBasis B, const double* boxC, int nbox,
                                                   const cx<double>* __restrict__ x, int ldx,
                                                   const TF* __restrict__ khat, int Q, TF kappa,
                                                   double w2e, int conjx, int nsplit, cx<TF>* __restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_box(blockIdx.x, nbox);
  if (b < 0) return;
  const int j0 = I.ptr[b], j1 = I.ptr[b + 1];
  const int npt = 7 * (j1 - j0);
  cx<TF>* dens = (cx<TF>*)smem;                              // [npt][5][RC]
  cx<TF>* part = dens + (size_t)npt * 5 * RC;                // [nsplit][Q][5][RC]
  TF* poff = (TF*)(part + (size_t)nsplit * Q * 5 * RC);      // [npt][3]
  const double* C = boxC + 3 * b;
  for (int p = threadIdx.x; p < npt; p += blockDim.x) {
    const int j = j0 + p / 7, i = p - 7 * (p / 7);
    const int t = I.tri[j];
    const double* P = G.P + 21 * t + 3 * i;
    const double w = G.W[7 * t + i];
    poff[3 * p + 0] = (TF)(P[0] - C[0]);
    poff[3 * p + 1] = (TF)(P[1] - C[1]);
    poff[3 * p + 2] = (TF)(P[2] - C[2]);
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      cx<double> J[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
      cx<double> D = mk(0.0, 0.0), sg = mk(0.0, 0.0);
      for (int k = 0; k < 3; ++k) {
        const int u = I.rwg[3 * j + k];
        if (u < 0) continue;
        cx<double> xv = x[(size_t)B.perm[u] * ldx + r];
        if (conjx) xv.im = -xv.im;
        const double s = I.rs[3 * j + k];
        const double* pv = G.V + 3 * I.rfv[3 * j + k];
        for (int d = 0; d < 3; ++d) J[d] = J[d] + (s * (P[d] - pv[d])) * xv;
        D = D + I.rd[3 * j + k] * xv;
      }
      const int up = I.pulse[j];
      if (up >= 0) {
        sg = x[(size_t)B.perm[up] * ldx + r];
        if (conjx) sg.im = -sg.im;
      }
      cx<TF>* dp = dens + (size_t)p * 5 * RC;
      for (int d = 0; d < 3; ++d) dp[d * RC + r] = mk((TF)(w * J[d].re), (TF)(w * J[d].im));
      dp[3 * RC + r] = mk((TF)(w * sg.re), (TF)(w * sg.im));
      cx<double> uu = D + w2e * sg;
      dp[4 * RC + r] = mk((TF)(w * uu.re), (TF)(w * uu.im));
    }
  }
  __syncthreads();
  constexpr int ncol = 5 * RC;
  if (threadIdx.x < nsplit * Q) {
    const int q = threadIdx.x % Q, part_id = threadIdx.x / Q;
    const TF kx = kappa * khat[3 * q], ky = kappa * khat[3 * q + 1], kz = kappa * khat[3 * q + 2];
    cx<TF> acc[ncol];
#pragma unroll
    for (int c = 0; c < ncol; ++c) acc[c] = mk<TF>(0, 0);
    for (int p = part_id; p < npt; p += nsplit) {
      const TF th = kx * poff[3 * p] + ky * poff[3 * p + 1] + kz * poff[3 * p + 2];
      cx<TF> d[ncol];
      const cx<TF>* dp = dens + (size_t)p * ncol;
#pragma unroll
      for (int c = 0; c < ncol; ++c) d[c] = dp[c];
      TF sn, cs;
      phase<TF, NT>(th, &sn, &cs);
      const cx<TF> e = mk(cs, -sn);
#pragma unroll
      for (int c = 0; c < ncol; ++c) cfma(acc[c], d[c], e);
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
// Child -> parent shift:  S_p(q) = sum_c exp(-i kappa_p khat_q.(C_c - C_p))
//                                   * sum_q' F[q][q'] S_c(q').
// Two passes.  k_child_filter: one workgroup per child stages the child's
// pattern in LDS (one coalesced copy) and one thread per (q, RHS) applies the
// filter row F[q][.] (read as Ft[q'][q], coalesced over q) to all five
// components, then the child's phase; the result goes to a per-child
// buffer.  k_child_sum: one thread per (parent, q, component, RHS) adds its
// children in Morton order (fixed order, no atomics).
// ---------------------------------------------------------------------------
template <typename TF>
__global__ void __launch_bounds__(128) k_child_filter(DevLevel Lc, const cx<TF>* __restrict__ Sc,
                                                      cx<TF>* __restrict__ Y, const TF* __restrict__ Ft,
                                                      const cx<TF>* __restrict__ ph, int Q, int R) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<TF>* Ss = (cx<TF>*)smem;  // [Q][5R]
  const int c = blockIdx.x;
  const int ncol = 5 * R;
  const int n = Q * ncol;
  const cx<TF>* src = Sc + (size_t)c * n;
  for (int e = threadIdx.x; e < n; e += blockDim.x) Ss[e] = src[e];
  __syncthreads();
  const cx<TF>* phc = ph + (size_t)Lc.octant[c] * Q;
  for (int e = threadIdx.x; e < Q * R; e += blockDim.x) {
    const int q = e / R, r = e - q * R;
    cx<TF> s[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) s[k] = mk<TF>(0, 0);
#pragma unroll 4
    for (int qq = 0; qq < Q; ++qq) {
      const TF f = Ft[(size_t)qq * Q + q];
      const cx<TF>* v = Ss + (size_t)qq * ncol + r;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const cx<TF> w = v[k * R];
        s[k].re = fma(f, w.re, s[k].re);
        s[k].im = fma(f, w.im, s[k].im);
      }
    }
    const cx<TF> pc = phc[q];
    cx<TF>* o = Y + (size_t)c * n + (size_t)q * ncol + r;
#pragma unroll
    for (int k = 0; k < 5; ++k) o[k * R] = pc * s[k];
  }
}

template <typename TF>
__global__ void __launch_bounds__(256) k_child_sum(DevLevel Lp, const cx<TF>* __restrict__ Y,
                                                   cx<TF>* __restrict__ Sp, int n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)Lp.nb * n) return;
  const int p = (int)(e / n), i = (int)(e - (int64_t)p * n);
  cx<TF> acc = mk<TF>(0, 0);
  for (int c = Lp.child_ptr[p]; c < Lp.child_ptr[p + 1]; ++c) acc = acc + Y[(size_t)c * n + i];
  Sp[e] = acc;
}

// ---------------------------------------------------------------------------
// Translation at one level, fused with the parent -> child shift of the
// parent's incoming pattern:
//   G_b(q) = sum_{b' in IL(b)} T_{off(b,b')}(q) S_b'(q)
//          + sum_q' F_p[q'][q] exp(+i kappa_p khat_q'.(C_b - C_p)) G_p(q').
// The translation is a gather (no atomics): the workgroup of box b reads its
// interaction list's patterns.
// ---------------------------------------------------------------------------
template <typename TF>
__global__ void __launch_bounds__(256) k_translate(DevLevel Lv, const cx<TF>* __restrict__ S,
                                                   const cx<TF>* __restrict__ T, cx<TF>* __restrict__ Gout,
                                                   int has_parent, const cx<TF>* __restrict__ Gp,
                                                   const TF* __restrict__ Fp, const cx<TF>* __restrict__ php,
                                                   int Q, int R) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<TF>* H = (cx<TF>*)smem;  // [Q][5R]
  const int b = xcd_box(blockIdx.x, Lv.nb);
  if (b < 0) return;
  const int ncol = 5 * R;
  const int n = Q * ncol;
  if (has_parent) {
    const int p = Lv.parent[b], oct = Lv.octant[b];
    const cx<TF>* g = Gp + (size_t)p * n;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      const int q = e / ncol;
      H[e] = conj(php[oct * Q + q]) * g[e];
    }
    __syncthreads();
  }
  const int i0 = Lv.il_ptr[b], i1 = Lv.il_ptr[b + 1];
  for (int e = threadIdx.x; e < Q * R; e += blockDim.x) {
    const int q = e / R, r = e - q * R;
    cx<TF> acc[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k] = mk<TF>(0, 0);
#pragma unroll 4
    for (int it = i0; it < i1; ++it) {
      const int src = Lv.il_src[it], off = Lv.il_off[it];
      const cx<TF> t = T[(size_t)off * Q + q];
      const cx<TF>* sv = S + (size_t)src * n + (size_t)q * ncol + r;
#pragma unroll
      for (int k = 0; k < 5; ++k) cfma(acc[k], t, sv[k * R]);
    }
    if (has_parent) {
#pragma unroll 4
      for (int qq = 0; qq < Q; ++qq) {
        const TF f = Fp[(size_t)qq * Q + q];
        const cx<TF>* h = H + (size_t)qq * ncol + r;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const cx<TF> v = h[k * R];
          acc[k].re = fma(f, v.re, acc[k].re);
          acc[k].im = fma(f, v.im, acc[k].im);
        }
      }
    }
    cx<TF>* o = Gout + (size_t)b * n + (size_t)q * ncol + r;
#pragma unroll
    for (int k = 0; k < 5; ++k) o[k * R] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// Reception at the finest level and join with the near-field partial sums.
// Per quadrature point the incoming field
//   fld(r_i) = W_i sum_q exp(+i kappa khat_q.(r_i - C_box)) G(q)
// is formed; then every unknown of the box takes its testing integral:
//   RWG:   y += mu0 s (r_i - p).fld_J + d fld_sigma   (both halves)
//   pulse: y += fld_u,
// adds its near-field partial sums in a fixed order, and is written to the
// canonical position (conjugated for the adjoint).
// ---------------------------------------------------------------------------
template <typename TF, typename TN, int RC, int NT>
__global__ void __launch_bounds__(256) k_receive(DevGeo G, DevInc I, DevBasis B, DevNear NB,
                                                 const double* boxC, int nbox, const cx<TF>* __restrict__ Gin,
                                                 const TF* __restrict__ khat, int Q, TF kappa,
                                                 const cx<TN>* __restrict__ part, int flags,
                                                 cx<double>* __restrict__ y, int ldy) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_box(blockIdx.x, nbox);
  if (b < 0) return;
  const int j0 = I.ptr[b], j1 = I.ptr[b + 1];
  const int npt = 7 * (j1 - j0);
  constexpr int ncol = 5 * RC;
  const bool do_far = flags & 2, do_near = flags & 1, conj_out = flags & 4;
  cx<TF>* fld = (cx<TF>*)smem;                             // [npt][5][RC]
  cx<TF>* Gs = fld + (size_t)npt * ncol;                   // [Q][5][RC]
  TF* kh = (TF*)(Gs + (size_t)Q * ncol);                   // [Q][4] kappa * khat
  TF* poff = kh + 4 * Q;                                   // [npt][3]
  const double mu0 = 4.0e-7 * 3.14159265358979323846;
  if (do_far) {
    const double* C = boxC + 3 * b;
    const cx<TF>* g = Gin + (size_t)b * Q * ncol;
    for (int e = threadIdx.x; e < Q * ncol; e += blockDim.x) Gs[e] = g[e];
    for (int q = threadIdx.x; q < Q; q += blockDim.x) {
      kh[4 * q + 0] = kappa * khat[3 * q];
      kh[4 * q + 1] = kappa * khat[3 * q + 1];
      kh[4 * q + 2] = kappa * khat[3 * q + 2];
      kh[4 * q + 3] = 0;
    }
    for (int p = threadIdx.x; p < npt; p += blockDim.x) {
      const int j = j0 + p / 7, i = p - 7 * (p / 7);
      const double* P = G.P + 21 * I.tri[j] + 3 * i;
      poff[3 * p + 0] = (TF)(P[0] - C[0]);
      poff[3 * p + 1] = (TF)(P[1] - C[1]);
      poff[3 * p + 2] = (TF)(P[2] - C[2]);
    }
    __syncthreads();
    for (int p = threadIdx.x; p < npt; p += blockDim.x) {
      cx<TF> acc[ncol];
#pragma unroll
      for (int c = 0; c < ncol; ++c) acc[c] = mk<TF>(0, 0);
      const TF ox = poff[3 * p], oy = poff[3 * p + 1], oz = poff[3 * p + 2];
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
      const int j = j0 + p / 7, i = p - 7 * (p / 7);
      const TF w = (TF)G.W[7 * I.tri[j] + i];
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
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
          const int slot = I.uslot[2 * u + h];
          const int j = slot >> 2, k = slot & 3;
          const int t = I.tri[j];
          const double s = I.rs[3 * j + k], d = I.rd[3 * j + k];
          const double* pv = G.V + 3 * I.rfv[3 * j + k];
          const cx<TF>* fp = fld + (size_t)(j - j0) * 7 * ncol;
#pragma unroll 1
          for (int i = 0; i < 7; ++i) {
            const double* P = G.P + 21 * t + 3 * i;
            const cx<TF>* f = fp + (size_t)i * ncol;
            cx<double> a = mk(0.0, 0.0);
            for (int c = 0; c < 3; ++c) {
              double dd = mu0 * s * (P[c] - pv[c]);
              a.re += dd * (double)f[c * RC + r].re;
              a.im += dd * (double)f[c * RC + r].im;
            }
            a.re += d * (double)f[3 * RC + r].re;
            a.im += d * (double)f[3 * RC + r].im;
            val = val + a;
          }
        }
      } else {
        const int j = I.uslot[2 * u] >> 2;
        const cx<TF>* fp = fld + (size_t)(j - j0) * 7 * ncol;
        for (int i = 0; i < 7; ++i) {
          val.re += (double)fp[(size_t)i * ncol + 4 * RC + r].re;
          val.im += (double)fp[(size_t)i * ncol + 4 * RC + r].im;
        }
      }
    }
    if (do_near) {
      for (int k = NB.row_ptr[b]; k < NB.row_ptr[b + 1]; ++k) {
        const cx<TN> v = part[((size_t)NB.prow[k] + ul) * RC + r];
        val.re += (double)v.re;
        val.im += (double)v.im;
      }
      for (int k = NB.col_ptr[b]; k < NB.col_ptr[b + 1]; ++k) {
        const cx<TN> v = part[((size_t)NB.pcol[NB.col_blk[k]] + ul) * RC + r];
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
         (size_t)maxpt * 3 * tf_bytes + 16;
}
size_t receive_smem(int maxpt, int Q, int R, int RC, int tf_bytes) {
  (void)R;
  return (size_t)maxpt * 5 * RC * 2 * tf_bytes + (size_t)Q * 5 * RC * 2 * tf_bytes + (size_t)Q * 4 * tf_bytes +
         (size_t)maxpt * 3 * tf_bytes + 16;
}

template <typename TF, int RC, int NT>
static void agg_launch(const DevGeo& G, const DevInc& I, const DevBasis& B, const double* boxC, int nb, int maxpt,
                       const void* x, int ldx, const void* khat, int Q, double kappa, double w2e, int conjx,
                       int nsplit, void* S, hipStream_t st) {
  size_t sm = aggregate_smem(maxpt, Q, nsplit, RC, sizeof(TF));
  hipLaunchKernelGGL((k_aggregate<TF, RC, NT>), dim3(xcd_grid(nb)), dim3(256), sm, st, G, I, B, boxC, nb,
                     (const cx<double>*)x, ldx, (const TF*)khat, Q, (TF)kappa, w2e, conjx, nsplit, (cx<TF>*)S);
}

template <typename TF>
hipError_t launch_aggregate(const DevGeo& G, const DevInc& I, const DevBasis& B, const double* boxC, int nb,
                            int maxpt, const void* x, int ldx, int R, const void* khat, int Q, double kappa,
                            double w2e, int conjx, int nsplit, int phase_mode, void* S, hipStream_t st) {
  constexpr int NS = sizeof(TF) == 8 ? 5 : 4, NL = sizeof(TF) == 8 ? 9 : 6;
  if (R != 1 && R != 2 && R != 4) return hipErrorInvalidValue;
#define AGG(RC_, NT_) agg_launch<TF, RC_, NT_>(G, I, B, boxC, nb, maxpt, x, ldx, khat, Q, kappa, w2e, conjx, nsplit, S, st)
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

template <typename TF>
hipError_t launch_shift_up(const DevLevel& Lp, const DevLevel& Lc, const void* Sc, void* Sp, const void* Ft,
                           const void* ph, int Q, int R, void* Ywork, hipStream_t st) {
  const int n = Q * 5 * R;
  hipLaunchKernelGGL(k_child_filter<TF>, dim3(Lc.nb), dim3(128), (size_t)n * 2 * sizeof(TF), st, Lc,
                     (const cx<TF>*)Sc, (cx<TF>*)Ywork, (const TF*)Ft, (const cx<TF>*)ph, Q, R);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t m = (int64_t)Lp.nb * n;
  hipLaunchKernelGGL(k_child_sum<TF>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, Lp,
                     (const cx<TF>*)Ywork, (cx<TF>*)Sp, n);
  return hipGetLastError();
}

template <typename TF>
hipError_t launch_translate(const DevLevel& Lv, const void* S, const void* T, void* Gout, int has_parent,
                            const void* Gp, const void* Fp, const void* php, int Q, int R, hipStream_t st) {
  size_t sm = has_parent ? (size_t)Q * 5 * R * 2 * sizeof(TF) : 16;
  hipLaunchKernelGGL(k_translate<TF>, dim3(xcd_grid(Lv.nb)), dim3(256), sm, st, Lv, (const cx<TF>*)S, (const cx<TF>*)T,
                     (cx<TF>*)Gout, has_parent, (const cx<TF>*)Gp, (const TF*)Fp, (const cx<TF>*)php, Q, R);
  return hipGetLastError();
}

template <typename TF, typename TN, int RC, int NT>
static void rec_launch(const DevGeo& G, const DevInc& I, const DevBasis& B, const DevNear& NB, const double* boxC,
                       int nb, int maxpt, const void* Gin, const void* khat, int Q, double kappa, const void* part,
                       int flags, void* y, int ldy, hipStream_t st) {
  size_t sm = receive_smem(maxpt, Q, RC, RC, sizeof(TF));
  hipLaunchKernelGGL((k_receive<TF, TN, RC, NT>), dim3(xcd_grid(nb)), dim3(256), sm, st, G, I, B, NB, boxC, nb,
                     (const cx<TF>*)Gin, (const TF*)khat, Q, (TF)kappa, (const cx<TN>*)part, flags,
                     (cx<double>*)y, ldy);
}

template <typename TF, typename TN>
hipError_t launch_receive(const DevGeo& G, const DevInc& I, const DevBasis& B, const DevNear& NB,
                          const double* boxC, int nb, int maxpt, const void* Gin, const void* khat, int Q,
                          double kappa, const void* part, int R, int flags, int phase_mode, void* y, int ldy,
                          hipStream_t st) {
  constexpr int NS = sizeof(TF) == 8 ? 5 : 4, NL = sizeof(TF) == 8 ? 9 : 6;
  if (R != 1 && R != 2 && R != 4) return hipErrorInvalidValue;
#define REC(RC_, NT_) \
  rec_launch<TF, TN, RC_, NT_>(G, I, B, NB, boxC, nb, maxpt, Gin, khat, Q, kappa, part, flags, y, ldy, st)
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
  template hipError_t launch_aggregate<TF>(const DevGeo&, const DevInc&, const DevBasis&, const double*, int, \
                                           int, const void*, int, int, const void*, int, double, double, int, \
                                           int, int, void*, hipStream_t);                                              \
  template hipError_t launch_shift_up<TF>(const DevLevel&, const DevLevel&, const void*, void*, const void*,  \
                                          const void*, int, int, void*, hipStream_t);                        \
  template hipError_t launch_translate<TF>(const DevLevel&, const void*, const void*, void*, int, const void*, \
                                           const void*, const void*, int, int, hipStream_t);                 \
  template hipError_t launch_permute_in<TF>(const void*, int, const int32_t*, int, int, int, void*,           \
                                            hipStream_t);
INST_F(float)
INST_F(double)
template hipError_t launch_receive<float, float>(const DevGeo&, const DevInc&, const DevBasis&, const DevNear&, const double*, int, int, const void*, const void*, int, double, const void*, int, int, int, void*, int, hipStream_t);
template hipError_t launch_receive<double, float>(const DevGeo&, const DevInc&, const DevBasis&, const DevNear&, const double*, int, int, const void*, const void*, int, double, const void*, int, int, int, void*, int, hipStream_t);
template hipError_t launch_receive<float, double>(const DevGeo&, const DevInc&, const DevBasis&, const DevNear&, const double*, int, int, const void*, const void*, int, double, const void*, int, int, int, void*, int, hipStream_t);
template hipError_t launch_receive<double, double>(const DevGeo&, const DevInc&, const DevBasis&, const DevNear&, const double*, int, int, const void*, const void*, int, double, const void*, int, int, int, void*, int, hipStream_t);

}  // namespace pie
