// Far field of the MLFMA (Section 3): radiation patterns and aggregation,
// diagonal translation with the scaled plane waves of Eq. (4) and the
// modified translation function of Eq. (5), disaggregation and reception.
//
// Pattern layout (outgoing S and incoming G of every level), box-major;
// c in {Jx, Jy, Jz, sigma, u}, u = div J + w^2 eps0 sigma, W = the RHS
// columns of the pass:
//   batched passes (W >= TB_MIN_COLS), sample-major:
//     P[((box * Q + q) * W + r) * 5 + c]
//   narrow passes, column-major:
//     P[((box * W + r) * Q + q) * 5 + c]
// Batched, the W x 5 values of one (box, sample) are one contiguous run: the
// translation gathers such runs (about as many times per box as its
// interaction list is long) and the shifts take blocks of them as GEMM
// columns.  Narrow, a box's Q x 5 values of one column are one run, which
// the sample lanes of the single-column kernels gather.  At W = 1 the two
// coincide.
#include <algorithm>

#include "device.h"
#include "kernels.h"

namespace pie {

typedef double f64x4 __attribute__((ext_vector_type(4)));  // v_mfma_f64 accumulator
constexpr int TSET_MAX = 8;  // levels per multi-level translation launch
constexpr int TB_MIN_COLS = 16;  // batched passes: W >= TB_MIN_COLS columns

// Strides (complex elements) of the pattern value (box, q, r, c) of a pass
// of W columns: box * Q * W * 5 + q * qs + r * rs + c.
struct PatStride {
  int qs, rs;
};
__host__ __device__ __forceinline__ PatStride pat_stride(int Q, int W) {
  return W >= TB_MIN_COLS ? PatStride{5 * W, 5} : PatStride{5, 5 * Q};
}

// ---------------------------------------------------------------------------
// Finest-level radiation patterns through per-incidence moments.  For a
// (box, triangle) incidence j with quadrature points r_i, weights W_i and
// o_i = r_i - C_box, the moment table holds (set-up, FP64 phases)
//   M0_j(q) = sum_i W_i e_i(q),   M1_j(q) = sum_i W_i o_i e_i(q),
//   e_i(q) = exp(-i kappa khat_q . o_i).
// The sample set is symmetric under khat -> -khat with the antipode of every
// sample q >= Qh among the first Qh, so M(q) = conj M(anti[q]) and only the
// first Qh samples are stored (Qh = Q/2; Qh = Q with anti[q] = q otherwise).
// An RWG half s (r - p) on the triangle radiates s (M1 - (p - C) M0); the
// scalar sources of the triangle radiate from its home incidence only (the
// box of its centroid): sigma = x_A and u = div J + w^2 eps0 x_A, with div J
// summed over all the RWG functions on the triangle, wherever they live.
// So with the incidence coefficients
//   a = sum_k x_k s_k,  b = sum_k x_k s_k (p_k - C)   (the box's RWG halves),
//   xp = x_A, cu = u     (home incidence; 0 otherwise)
// the box patterns are
//   S_J(q) += a M1 - b M0,  S_sigma(q) += xp M0,  S_u(q) += cu M0.
// ---------------------------------------------------------------------------
// u of triangle t for column col (conjugated input for the adjoint).
__device__ __forceinline__ cx<double> tri_u(const DevTriDiv& td, const cx<double>* __restrict__ x, int ldx,
                                            int col, int t, cx<double> xa, double w2e, int conjx) {
  cx<double> u = w2e * xa;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int e = td.e[3 * t + k];
    if (e >= 0) {
      cx<double> v = x[(size_t)e * ldx + col];
      if (conjx) v.im = -v.im;
      u = u + td.d[3 * t + k] * v;
    }
  }
  return u;
}

template <typename TF>
__global__ void __launch_bounds__(128) k_moments(const double* __restrict__ pw, const double* __restrict__ khat,
                                                 int Qh, double kappa, cx<TF>* __restrict__ M) {
  const int j = blockIdx.x;
  const double* p = pw + 28 * (size_t)j;
  double o[7][3], w[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) {
#pragma unroll
    for (int c = 0; c < 3; ++c) o[i][c] = p[4 * i + c];
    w[i] = p[4 * i + 3];
  }
  for (int q = threadIdx.x; q < Qh; q += blockDim.x) {
    const double kx = kappa * khat[3 * q], ky = kappa * khat[3 * q + 1], kz = kappa * khat[3 * q + 2];
    cx<double> m0 = mk(0.0, 0.0), m1[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      double sn, cs;
      sincos(kx * o[i][0] + ky * o[i][1] + kz * o[i][2], &sn, &cs);
      const cx<double> e = mk(w[i] * cs, -w[i] * sn);
      m0 = m0 + e;
#pragma unroll
      for (int c = 0; c < 3; ++c) m1[c] = m1[c] + o[i][c] * e;
    }
    cx<TF>* out = M + ((size_t)j * Qh + q) * 4;
    out[0] = mk((TF)m0.re, (TF)m0.im);
#pragma unroll
    for (int c = 0; c < 3; ++c) out[1 + c] = mk((TF)m1[c].re, (TF)m1[c].im);
  }
}

// Workgroup = one finest box; the W right-hand-side columns are taken in
// groups of RC.  Stage 1: thread per (incidence, column) forms the
// coefficients (a, -b, xp, cu) in LDS.  Stage 2: thread (g, s) adds the
// incidences j = g (mod nsplit) in order for the stored sample s and its
// antipode, two (FP64) or four (FP32) incidences' moments in flight (the
// box's moments are re-read from L2 for later groups); stage 3 adds the
// nsplit slices in a fixed order.  Each column's arithmetic is the same for
// any W and RC.
template <typename TF, int RC>
__global__ void __launch_bounds__(256) k_aggregate(DevInc I, int nbox, const cx<double>* __restrict__ x, int ldx,
                                                   const cx<TF>* __restrict__ M, const int32_t* __restrict__ anti,
                                                   int Q, int Qh, double w2e, int conjx, int nsplit, int W,
                                                   cx<TF>* __restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_box(blockIdx.x, nbox);
  if (b < 0) return;
  const int j0 = I.ptr[b], ni = I.ptr[b + 1] - j0;
  const PatStride ps = pat_stride(Q, W);
  constexpr int ncol = 5 * RC;
  cx<TF>* cf = (cx<TF>*)smem;                      // [ni][6][RC]: a, -bx, -by, -bz, xp, cu
  cx<TF>* part = cf + (size_t)ni * 6 * RC;         // [nsplit - 1][Q][5][RC]
  int32_t* pair = (int32_t*)(part + (size_t)(nsplit - 1) * Q * ncol);  // [Qh] antipode of a stored sample
  const bool paired = Qh < Q;
  const int g = threadIdx.x / Qh, sq = threadIdx.x - g * Qh;  // group, stored sample
  const bool act = g < nsplit;
  for (int q = Qh + threadIdx.x; q < Q; q += blockDim.x) pair[anti[q]] = q;
  for (int c0 = 0; c0 < W; c0 += RC) {
    if (c0 > 0) __syncthreads();
    for (int e = threadIdx.x; e < ni * RC; e += blockDim.x) {
      const int jl = e / RC, r = e - jl * RC;
      const size_t j = (size_t)(j0 + jl);
      int xc[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) xc[k] = c0 + r < W ? I.xc[4 * j + k] : -1;
      double sv[3], pv[3][3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sv[k] = I.rs[3 * j + k];
#pragma unroll
        for (int c = 0; c < 3; ++c) pv[k][c] = I.pv[9 * j + 3 * k + c];
      }
      cx<double> xv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xv[k] = xc[k] >= 0 ? x[(size_t)xc[k] * ldx + c0 + r] : mk(0.0, 0.0);
        if (conjx) xv[k].im = -xv[k].im;
      }
      cx<double> a = mk(0.0, 0.0), bb[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        a = a + sv[k] * xv[k];
#pragma unroll
        for (int c = 0; c < 3; ++c) bb[c] = bb[c] + (sv[k] * pv[k][c]) * xv[k];
      }
      const cx<double> cu =
          xc[3] >= 0 ? tri_u(I.td, x, ldx, c0 + r, xc[3] - I.td.ne, xv[3], w2e, conjx) : mk(0.0, 0.0);
      cx<TF>* o = cf + (size_t)jl * 6 * RC + r;
      o[0] = mk((TF)a.re, (TF)a.im);
#pragma unroll
      for (int c = 0; c < 3; ++c) o[(1 + c) * RC] = mk((TF)-bb[c].re, (TF)-bb[c].im);
      o[4 * RC] = mk((TF)xv[3].re, (TF)xv[3].im);
      o[5 * RC] = mk((TF)cu.re, (TF)cu.im);
    }
    __syncthreads();
    // sample sq takes M(sq), its antipode pair[sq] takes conj M(sq): every
    // stored moment is loaded once and used twice
    cx<TF> acc[ncol], acc2[ncol];
#pragma unroll
    for (int c = 0; c < ncol; ++c) acc[c] = acc2[c] = mk<TF>(0, 0);
    auto add = [&](cx<TF>(&ac)[ncol], const cx<TF>(&mm)[4], const cx<TF>* c6) {
#pragma unroll
      for (int r = 0; r < RC; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cfma(ac[c * RC + r], c6[r], mm[1 + c]);
          cfma(ac[c * RC + r], c6[(1 + c) * RC + r], mm[0]);
        }
        cfma(ac[3 * RC + r], c6[4 * RC + r], mm[0]);
        cfma(ac[4 * RC + r], c6[5 * RC + r], mm[0]);
      }
    };
    const int q2 = act && paired ? pair[sq] : 0;
    if (act) {
      constexpr int U = sizeof(TF) == 8 ? 2 : 4;
      for (int jl = g; jl < ni; jl += U * nsplit) {
        cx<TF> m[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int jj = jl + u * nsplit;
          const cx<TF>* mp = M + ((size_t)(j0 + (jj < ni ? jj : jl)) * Qh + sq) * 4;
#pragma unroll
          for (int t = 0; t < 4; ++t) m[u][t] = mp[t];
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the incidences' loads in flight together
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int jj = jl + u * nsplit;
          if (jj < ni) {
            const cx<TF>* c6 = cf + (size_t)jj * 6 * RC;
            add(acc, m[u], c6);
            if (paired) {
              cx<TF> cm[4];
#pragma unroll
              for (int t = 0; t < 4; ++t) cm[t] = conj(m[u][t]);
              add(acc2, cm, c6);
            }
          }
        }
      }
      if (g > 0) {
        cx<TF>* pp = part + ((size_t)(g - 1) * Q + sq) * ncol;
#pragma unroll
        for (int c = 0; c < ncol; ++c) pp[c] = acc[c];
        if (paired) {
          cx<TF>* p2 = part + ((size_t)(g - 1) * Q + q2) * ncol;
#pragma unroll
          for (int c = 0; c < ncol; ++c) p2[c] = acc2[c];
        }
      }
    }
    __syncthreads();
    if (act && g == 0) {
      for (int h = 1; h < nsplit; ++h) {
        const cx<TF>* pp = part + ((size_t)(h - 1) * Q + sq) * ncol;
        const cx<TF>* p2 = part + ((size_t)(h - 1) * Q + q2) * ncol;
#pragma unroll
        for (int c = 0; c < ncol; ++c) {
          acc[c] = acc[c] + pp[c];
          if (paired) acc2[c] = acc2[c] + p2[c];
        }
      }
#pragma unroll
      for (int r = 0; r < RC; ++r)
        if (c0 + r < W) {
          cx<TF>* o = S + (size_t)b * Q * W * 5 + (size_t)sq * ps.qs + (size_t)(c0 + r) * ps.rs;
#pragma unroll
          for (int k = 0; k < 5; ++k) o[k] = acc[k * RC + r];
          if (paired) {
            cx<TF>* o2 = S + (size_t)b * Q * W * 5 + (size_t)q2 * ps.qs + (size_t)(c0 + r) * ps.rs;
#pragma unroll
            for (int k = 0; k < 5; ++k) o2[k] = acc2[k * RC + r];
          }
        }
    }
  }
}

// ---------------------------------------------------------------------------
// Batched FP64 aggregation on the matrix cores (W >= MA_COLS columns in a
// pass, paired samples).  For a box and a block of MA_COLS columns the
// patterns are complex GEMMs over the box's incidences j:
//   S_Jc = M1c a + M0 (-b_c),  S_sigma = M0 xp,  S_u = M0 cu
// (rows: the Qh stored samples s).  With A = M(s) = Ar + i Ai and the
// coefficient B = Br + i Bi, the real products P1 = Ar Br, P2 = Ai Bi,
// P3 = Ar Bi, P4 = Ai Br give S(s) = (P1 - P2, P3 + P4) and, since
// M(anti s) = conj M(s), S(anti s) = (P1 + P2, P3 - P4): every moment feeds
// two samples.  Wave w takes the row tiles w, w + 4, ...; a K step is four
// incidences; the coefficients of MA_JC incidences at a time are formed in
// LDS as in k_aggregate.  v_mfma_f64_16x16x4 operand layout as for the
// shifts.
// ---------------------------------------------------------------------------
constexpr int MA_COLS = 16;  // columns per workgroup
static_assert(MA_COLS >= TB_MIN_COLS, "the matrix-core aggregation writes sample-major patterns");
constexpr int MA_JC = 16;    // incidences per coefficient chunk (a multiple of 4)

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_maggregate(DevInc I, int nbox, const cx<double>* __restrict__ x, int ldx,
                                                    const cx<double>* __restrict__ M,
                                                    const int32_t* __restrict__ anti, int Q, int Qh, double w2e,
                                                    int conjx, int W, cx<double>* __restrict__ S) {
  __shared__ cx<double> cf[MA_JC][6][MA_COLS];  // a, -bx, -by, -bz, xp, cu
  __shared__ int32_t pair[256];
  const int b = xcd_box(blockIdx.x, nbox);
  if (b < 0) return;
  const int c0 = blockIdx.y * MA_COLS;
  const int j0 = I.ptr[b], ni = I.ptr[b + 1] - j0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, kq = lane >> 4, jl = lane & 15;
  const bool paired = Qh < Q;
  for (int q = Qh + threadIdx.x; q < Q; q += blockDim.x) pair[anti[q]] = q;
  __syncthreads();
  const int ntile = (Qh + 15) >> 4;
  for (int rt0 = 0; rt0 < ntile; rt0 += 4) {
    const int rt = rt0 + w;  // this wave's row tile (may be past the last one)
    const int s = rt * 16 + jl;
    const bool srow = rt < ntile && s < Qh;
    f64x4 acc[5][4];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int p = 0; p < 4; ++p) acc[k][p] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int jc = 0; jc < ni; jc += MA_JC) {
      const int nj = min(MA_JC, ni - jc);
      __syncthreads();  // previous chunk's coefficients consumed
      for (int e = threadIdx.x; e < MA_JC * MA_COLS; e += blockDim.x) {
        const int jj = e / MA_COLS, r = e - jj * MA_COLS;
        cx<double> v[6];
        if (jj < nj && c0 + r < W) {
          const size_t j = (size_t)(j0 + jc + jj);
          cx<double> xv[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int xi = I.xc[4 * j + k];
            xv[k] = xi >= 0 ? x[(size_t)xi * ldx + c0 + r] : mk(0.0, 0.0);
            if (conjx) xv[k].im = -xv[k].im;
          }
          cx<double> a = mk(0.0, 0.0), bb[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double sv = I.rs[3 * j + k];
            a = a + sv * xv[k];
#pragma unroll
            for (int c = 0; c < 3; ++c) bb[c] = bb[c] + (sv * I.pv[9 * j + 3 * k + c]) * xv[k];
          }
          const int xp = I.xc[4 * j + 3];
          const cx<double> cu =
              xp >= 0 ? tri_u(I.td, x, ldx, c0 + r, xp - I.td.ne, xv[3], w2e, conjx) : mk(0.0, 0.0);
          v[0] = a;
#pragma unroll
          for (int c = 0; c < 3; ++c) v[1 + c] = mk(-bb[c].re, -bb[c].im);
          v[4] = xv[3];
          v[5] = cu;
        } else {
#pragma unroll
          for (int t = 0; t < 6; ++t) v[t] = mk(0.0, 0.0);
        }
#pragma unroll
        for (int t = 0; t < 6; ++t) cf[jj][t][r] = v[t];
      }
      __syncthreads();
      if (rt < ntile) {
        // moments of step k0 + 4 load while step k0 is multiplied
        auto load_m = [&](int k0, cx<double>(&m)[4]) {
          const int jj = k0 + kq;
          const bool ok = srow && jj < nj;
          const cx<double>* mp = M + ((size_t)(j0 + jc + (ok ? jj : 0)) * Qh + (ok ? s : 0)) * 4;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const cx<double> v = mp[t];
            m[t] = ok ? v : mk(0.0, 0.0);
          }
        };
        cx<double> mn[4];
        load_m(0, mn);
        for (int k0 = 0; k0 < nj; k0 += 4) {
          const int jj = k0 + kq;
          cx<double> m[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) m[t] = mn[t];
          if (k0 + 4 < nj) load_m(k0 + 4, mn);
          cx<double> bv[6];
#pragma unroll
          for (int t = 0; t < 6; ++t) bv[t] = cf[jj < MA_JC ? jj : 0][t][jl];
          // (moment, coefficient, component): M1c a -> Jc; M0 (-b_c) -> Jc; M0 xp -> sigma; M0 cu -> u
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int mi = t < 3 ? 1 + t : 0, bi = t < 3 ? 0 : t - 2, k = t < 3 ? t : (t < 6 ? t - 3 : t - 3);
            const cx<double> A = m[mi], B = bv[bi];
            acc[k][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.re, B.re, acc[k][0], 0, 0, 0);
            acc[k][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.im, B.im, acc[k][1], 0, 0, 0);
            acc[k][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.re, B.im, acc[k][2], 0, 0, 0);
            acc[k][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.im, B.re, acc[k][3], 0, 0, 0);
          }
        }
      }
    }
    // epilogue: lane holds rows s = 16 rt + kq + 4 v of column c0 + jl
    const int r = c0 + jl;
    if (rt < ntile && r < W) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int sv = rt * 16 + kq + 4 * v;
        if (sv < Qh) {
          cx<double>* o = S + (((size_t)b * Q + sv) * W + r) * 5;
#pragma unroll
          for (int k = 0; k < 5; ++k)
            o[k] = mk(acc[k][0][v] - acc[k][1][v], acc[k][2][v] + acc[k][3][v]);
          if (paired) {
            cx<double>* o2 = S + (((size_t)b * Q + pair[sv]) * W + r) * 5;
#pragma unroll
            for (int k = 0; k < 5; ++k)
              o2[k] = mk(acc[k][0][v] + acc[k][1][v], acc[k][2][v] - acc[k][3][v]);
          }
        }
      }
    }
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
__device__ __forceinline__ bool shift_item(int ngroup, int ntile, int R, int rows, ShiftItem& it) {
  const int per = (ngroup + 7) >> 3, w = blockIdx.x, x = w & 7, j = w >> 3;
  const int sub = ntile * R, gl = j / sub, rem = j - gl * sub;
  it.g = x * per + gl;
  it.q0 = (rem / R) * rows;
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
  if (!shift_item(Lp.nug, ntile, R, SQT, it)) return;
  const int q0 = it.q0, r = it.r;
  const PatStride ps = pat_stride(Q, R);
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
    const cx<TF>* s = Sc + (size_t)c * Q * R * 5 + (size_t)r * ps.rs + k;
    shift_mac(Fs, qa, qb, [&](int qq) { return s[(size_t)qq * ps.qs]; }, acc);
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
    Sp[(size_t)p * Q * R * 5 + (size_t)(q0 + i) * ps.qs + (size_t)r * ps.rs + kk] = v;
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
  if (!shift_item(ng, ntile, R, SQT, it)) return;
  const int q0 = it.q0, r = it.r;
  const PatStride ps = pat_stride(Q, R);
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
    const cx<TF>* gp = Gp + (size_t)Lc.parent[c] * Q * R * 5 + (size_t)r * ps.rs + k;
    const cx<TF>* pc = ph + (size_t)Lc.octant[c] * Q;
    shift_mac(Fs, qa, qb, [&](int qq) { return conj(pc[qq]) * gp[(size_t)qq * ps.qs]; }, acc);
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
    cx<TF>* o = Gc + (size_t)c * Q * R * 5 + (size_t)q0 * ps.qs + (size_t)r * ps.rs + k;
#pragma unroll
    for (int i = 0; i < SQT; ++i)
      if (i < nq) o[(size_t)i * ps.qs] = o[(size_t)i * ps.qs] + acc[i];
  }
}

// ---------------------------------------------------------------------------
// FP64 shifts on the matrix cores.  The filter product is a real GEMM
//   D[q][col] = sum_q' F[q][q'] B[q'][col]
// in v_mfma_f64_16x16x4 tiles.  A workgroup owns MS_ROWS = 32 output samples
// and MS_COLS = 128 real columns; wave w holds the 2 x 2 tiles of rows
// 0..31 and columns 32w .. 32w+31 (tiles past the last column are skipped).
// The filter block is staged in LDS (zeros pad Q to whole tiles and K
// steps) and B is read from the pattern array eight K steps at a time.
// In batched passes the columns are a block of a sample row (W x 10 values):
// upward, one child's rows, the children phased and summed in registers;
// downward, the parent's rows phased for one child as they are loaded, the
// result added to the child's incoming pattern.  Narrow passes take as
// columns (child, component, re/im) of a group of up to SHIFT_GROUP children
// for one RHS column.
// Operand layout of v_mfma_f64_16x16x4 (64 lanes): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register v of lane l is
// D[l / 16 + 4 v][l % 16].
// ---------------------------------------------------------------------------
constexpr int MS_ROWS = 32;
constexpr int MS_COLS = 128;
constexpr int MS_MIN_ITEMS = 256;  // (group, row block) items for the matrix-core path
constexpr int MS_RCH = 8;          // RHS columns per workgroup (the filter block is staged once for them)
static_assert(SHIFT_GROUP * 10 <= MS_COLS, "shift group exceeds the GEMM columns");

__host__ __device__ inline size_t mshift_smem(int Q) {
  const int kp = (Q + 3) & ~3;
  return (size_t)std::max(kp, MS_COLS) * MS_ROWS * sizeof(double);
}

// Fs[k][i] = table[k][q0 + i] (input sample k, output sample q0 + i), zero
// outside the Q x Q table.
__device__ __forceinline__ void mshift_stage(const double* __restrict__ tab, double* Fs, int Q, int q0) {
  const int kp = (Q + 3) & ~3;
  for (int e = threadIdx.x; e < kp * MS_ROWS; e += blockDim.x) {
    const int k = e / MS_ROWS, i = e - k * MS_ROWS;
    Fs[e] = k < Q && q0 + i < Q ? tab[(size_t)k * Q + q0 + i] : 0.0;
  }
}

// acc[t][ct] += A_t B_ct over all K, A from Fs; B(ct, k) = value(ct, k,
// fetch(ct, k)) for k < Q, 0 beyond.  fetch issues the (unconditional,
// in-bounds) global loads; batches of KU K steps are double-buffered in
// registers, so the next batch is in flight while this one is multiplied.
// pre() stages Fs (and what else the epilogue needs) after the first batch
// is issued.
// col_ok[ct]: the wave's column tile ct holds some column of the group.
template <int KU, typename T, typename FE, typename VA, typename PRE>
__device__ __forceinline__ void mshift_gemm(const double* Fs, int Q, const bool (&col_ok)[2], FE fetch, VA value,
                                            PRE pre, f64x4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, kq = lane >> 4, jl = lane & 15;
  const int kp = (Q + 3) & ~3, kb = 4 * KU, nbat = (kp + kb - 1) / kb;
  T b0[KU][2], b1[KU][2];
  auto get = [&](T (&bv)[KU][2], int k0) {
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) bv[u][ct] = fetch(ct, min(k0 + 4 * u + kq, Q - 1));
  };
  auto mul = [&](const T (&bv)[KU][2], int k0) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      if (k0 + 4 * u >= kp) break;
      const int k = k0 + 4 * u + kq;
      const double a0 = Fs[k * MS_ROWS + jl], a1 = Fs[k * MS_ROWS + 16 + jl];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
        if (col_ok[ct]) {
          const double bb = k < Q ? value(ct, k, bv[u][ct]) : 0.0;
          acc[0][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bb, acc[0][ct], 0, 0, 0);
          acc[1][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bb, acc[1][ct], 0, 0, 0);
        }
    }
  };
  get(b0, 0);
  pre();  // LDS staging, overlapped with the first batch's loads; ends in a barrier
  for (int n = 0; n < nbat; n += 2) {
    if (n + 1 < nbat) get(b1, (n + 1) * kb);
    mul(b0, n * kb);
    if (n + 1 >= nbat) break;
    if (n + 2 < nbat) get(b0, (n + 2) * kb);
    mul(b1, (n + 1) * kb);
  }
}

// The same product with A read from the global filter table (rows q0 ..
// q0 + 31 of the output, clamped to the table; rows past Q are never
// stored, and K steps past Q meet a zero B), so that the workgroup keeps no
// filter block in LDS; A is double-buffered with B.
template <int KU, typename T, typename FE, typename VA, typename PRE>
__device__ __forceinline__ void mshift_gemm_ga(const double* __restrict__ tab, int q0, int Q,
                                               const bool (&col_ok)[2], FE fetch, VA value, PRE pre,
                                               f64x4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, kq = lane >> 4, jl = lane & 15;
  const int kp = (Q + 3) & ~3, kb = 4 * KU, nbat = (kp + kb - 1) / kb;
  const int ra = min(q0 + jl, Q - 1), rb = min(q0 + 16 + jl, Q - 1);
  T b0[KU][2], b1[KU][2];
  double a0s[KU][2], a1s[KU][2];
  auto get = [&](T (&bv)[KU][2], double (&av)[KU][2], int k0) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = min(k0 + 4 * u + kq, Q - 1);
      av[u][0] = tab[(size_t)k * Q + ra];
      av[u][1] = tab[(size_t)k * Q + rb];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) bv[u][ct] = fetch(ct, k);
    }
  };
  auto mul = [&](const T (&bv)[KU][2], const double (&av)[KU][2], int k0) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      if (k0 + 4 * u >= kp) break;
      const int k = k0 + 4 * u + kq;
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
        if (col_ok[ct]) {
          const double bb = k < Q ? value(ct, k, bv[u][ct]) : 0.0;
          acc[0][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][0], bb, acc[0][ct], 0, 0, 0);
          acc[1][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][1], bb, acc[1][ct], 0, 0, 0);
        }
    }
  };
  get(b0, a0s, 0);
  pre();
  for (int n = 0; n < nbat; n += 2) {
    if (n + 1 < nbat) get(b1, a1s, (n + 1) * kb);
    mul(b0, a0s, n * kb);
    if (n + 1 >= nbat) break;
    if (n + 2 < nbat) get(b0, a0s, (n + 2) * kb);
    mul(b1, a1s, (n + 1) * kb);
  }
}

// acc -> Ds[row][col]
__device__ __forceinline__ void mshift_store(const f64x4 (&acc)[2][2], double* Ds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Ds[(t * 16 + (lane >> 4) + 4 * v) * MS_COLS + w * 32 + ct * 16 + (lane & 15)] = acc[t][ct][v];
}

// Upward shift on the matrix cores for narrow passes (W < TB_MIN_COLS): the
// GEMM columns are (child, component, re/im) of the children of a group of
// parents (at most SHIFT_GROUP children) for one RHS column; the result goes
// through LDS, where each child row is phased and the children of a parent
// are added in Morton order.  The filter rows are read from the global table
// (no filter block in LDS).
__global__ void __launch_bounds__(256, 3) k_mshift_up_groups(DevLevel Lp, DevLevel Lc, const cx<double>* __restrict__ Sc,
                                                   cx<double>* __restrict__ Sp, const double* __restrict__ Ft,
                                                   const cx<double>* __restrict__ ph, int Q, int R, int ntile,
                                                   int nchunk) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* Ds = (double*)smem;                                            // [MS_ROWS][MS_COLS] result
  cx<double>* phs = (cx<double>*)(Ds + MS_ROWS * MS_COLS);               // [child][row] output phases
  int32_t* cps = (int32_t*)(phs + SHIFT_GROUP * MS_ROWS);                // child ranges of the parents
  ShiftItem it;
  if (!shift_item(Lp.nug, ntile, nchunk, MS_ROWS, it)) return;
  const int q0 = it.q0;
  const int nq = min(MS_ROWS, Q - q0);
  const int p0 = Lp.ug_ptr[it.g], p1 = Lp.ug_ptr[it.g + 1];
  const int c0 = Lp.child_ptr[p0], c1 = Lp.child_ptr[p1];
  const int nch = c1 - c0, ncols = 10 * nch, np = p1 - p0;
  const int w = threadIdx.x >> 6, jl = threadIdx.x & 15;
  const double* S = (const double*)Sc;
  const int r0 = it.r * MS_RCH, r1 = min(R, r0 + MS_RCH);
  for (int r = r0; r < r1; ++r) {
    size_t base[2];
    bool col_ok[2], valid[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int cbase = w * 32 + ct * 16, col = cbase + jl;
      col_ok[ct] = cbase < ncols;
      valid[ct] = col < ncols;
      const int ci = col / 10, rem = col - ci * 10;
      base[ct] = valid[ct] ? (((size_t)(c0 + ci) * R + r) * Q) * 10 + rem : 0;
    }
    f64x4 acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) acc[t][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
    mshift_gemm_ga<4, double>(
        Ft, q0, Q, col_ok, [&](int ct, int k) { return S[base[ct] + (size_t)k * 10]; },
        [&](int ct, int, double v) { return valid[ct] ? v : 0.0; },
        [&] {
          if (r == r0) {  // phases and child ranges, once for all columns
            for (int e = threadIdx.x; e < nch * nq; e += blockDim.x) {
              const int ci = e / nq, i = e - ci * nq;
              phs[ci * MS_ROWS + i] = ph[(size_t)Lc.octant[c0 + ci] * Q + q0 + i];
            }
            for (int e = threadIdx.x; e <= np; e += blockDim.x) cps[e] = Lp.child_ptr[p0 + e] - c0;
          }
          __syncthreads();  // also: the previous column's result is consumed
        },
        acc);
    mshift_store(acc, Ds);
    __syncthreads();
    const int m = np * nq * 5;
    for (int e = threadIdx.x; e < m; e += blockDim.x) {
      const int pl = e / (nq * 5), rem = e - pl * nq * 5;
      const int i = rem / 5, kk = rem - i * 5;
      cx<double> v = mk(0.0, 0.0);
      for (int ci = cps[pl]; ci < cps[pl + 1]; ++ci) {
        const double* d = Ds + i * MS_COLS + ci * 10 + 2 * kk;
        v = v + phs[ci * MS_ROWS + i] * mk(d[0], d[1]);
      }
      Sp[(((size_t)(p0 + pl) * R + r) * Q + q0 + i) * 5 + kk] = v;
    }
  }
}

// Upward shift on the matrix cores for batched passes (W >= TB_MIN_COLS,
// sample-major outgoing patterns).  A workgroup owns one parent p, its
// output rows q0 .. q0 + 31 and a block of MS_COLS real columns n of a
// sample row (n = (RHS column, component, re/im), W x 10 values):
//   S_p[q][n] = sum_{children c, Morton order} ph_c(q) sum_k F[q][k] S_c[k][n]
// One child at a time: the filter product on the matrix cores (its B rows are
// the child's sample rows, 16 lanes reading 16 consecutive values), then the
// complex phase of the output row applied in registers (real and imaginary
// parts of a value sit in adjacent lanes) as the child is added.
__global__ void __launch_bounds__(256, 3) k_mshift_up(DevLevel Lp, DevLevel Lc, const cx<double>* __restrict__ Sc,
                                                   cx<double>* __restrict__ Sp, const double* __restrict__ Ft,
                                                   const cx<double>* __restrict__ ph, int Q, int R, int ntile,
                                                   int nnb) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* Fs = (double*)smem;                                              // filter block
  cx<double>* phs = (cx<double>*)(Fs + mshift_smem(Q) / sizeof(double));   // [8][MS_ROWS] output phases
  ShiftItem it;
  if (!shift_item(Lp.nb, ntile, nnb, MS_ROWS, it)) return;
  const int p = it.g, q0 = it.q0, nq = min(MS_ROWS, Q - q0);
  const int c0 = Lp.child_ptr[p], nch = Lp.child_ptr[p + 1] - c0;
  const int ncol = 10 * R, n0 = it.r * MS_COLS;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, jl = lane & 15;
  int col[2];
  bool col_ok[2], valid[2];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int cbase = n0 + w * 32 + ct * 16;
    col_ok[ct] = cbase < ncol;
    valid[ct] = cbase + jl < ncol;
    col[ct] = valid[ct] ? cbase + jl : 0;
  }
  mshift_stage(Ft, Fs, Q, q0);
  for (int e = threadIdx.x; e < nch * MS_ROWS; e += blockDim.x) {
    const int ci = e / MS_ROWS, i = e - ci * MS_ROWS;
    phs[e] = i < nq ? ph[(size_t)Lc.octant[c0 + ci] * Q + q0 + i] : mk(0.0, 0.0);
  }
  __syncthreads();
  f64x4 sum[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) sum[t][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int ci = 0; ci < nch; ++ci) {
    const double* S = (const double*)Sc + (size_t)(c0 + ci) * Q * ncol;
    f64x4 acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) acc[t][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
    mshift_gemm<4, double>(
        Fs, Q, col_ok, [&](int ct, int k) { return S[(size_t)k * ncol + col[ct]]; },
        [&](int ct, int, double v) { return valid[ct] ? v : 0.0; }, [] {}, acc);
    // result register v of lane l is row l / 16 + 4 v of tile (t, ct)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        if (!col_ok[ct]) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const cx<double> f = phs[ci * MS_ROWS + t * 16 + (lane >> 4) + 4 * v];
          const double mine = acc[t][ct][v], other = __shfl_xor(mine, 1);
          sum[t][ct][v] += f.re * mine + (lane & 1 ? f.im : -f.im) * other;
        }
      }
  }
  double* out = (double*)Sp + ((size_t)p * Q + q0) * ncol;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = t * 16 + (lane >> 4) + 4 * v;
        if (valid[ct] && i < nq) out[(size_t)i * ncol + col[ct]] = sum[t][ct][v];
      }
}

// Downward shift on the matrix cores for narrow passes (W < TB_MIN_COLS):
// columns (child, component, re/im) of SHIFT_GROUP consecutive children for
// one RHS column at a time; the epilogue adds to the incoming patterns
// straight from the accumulators.
__global__ void __launch_bounds__(256, 3) k_mshift_down_groups(DevLevel Lc, const cx<double>* __restrict__ Gp,
                                                     cx<double>* __restrict__ Gc, const double* __restrict__ F,
                                                     const cx<double>* __restrict__ ph, int Q, int R, int ntile,
                                                     int nchunk) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* Fs = (double*)smem;                                       // filter block
  cx<double>* phs = (cx<double>*)(Fs + mshift_smem(Q) / sizeof(double));  // [8][Q] phases
  const int ng = (Lc.nb + SHIFT_GROUP - 1) / SHIFT_GROUP;
  ShiftItem it;
  if (!shift_item(ng, ntile, nchunk, MS_ROWS, it)) return;
  const int q0 = it.q0;
  const int nq = min(MS_ROWS, Q - q0);
  const int c0 = it.g * SHIFT_GROUP, c1 = min(Lc.nb, c0 + SHIFT_GROUP);
  const int ncols = 10 * (c1 - c0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, jl = threadIdx.x & 15;
  const int r0 = it.r * MS_RCH, r1 = min(R, r0 + MS_RCH);
  for (int r = r0; r < r1; ++r) {
    const cx<double>* gp[2];
    int po[2];
    bool col_ok[2], valid[2], im[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int cbase = w * 32 + ct * 16, col = cbase + jl;
      col_ok[ct] = cbase < ncols;
      valid[ct] = col < ncols;
      const int ci = col / 10, rem = col - ci * 10;
      const int c = valid[ct] ? c0 + ci : c0;
      gp[ct] = Gp + (((size_t)Lc.parent[c] * R + r) * Q) * 5 + (rem >> 1);
      po[ct] = Lc.octant[c] * Q;
      im[ct] = rem & 1;
    }
    f64x4 acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) acc[t][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
    mshift_gemm<4, cx<double>>(
        Fs, Q, col_ok, [&](int ct, int k) { return gp[ct][(size_t)k * 5]; },
        [&](int ct, int k, const cx<double>& g) {
          const cx<double> v = conj(phs[po[ct] + k]) * g;
          return valid[ct] ? (im[ct] ? v.im : v.re) : 0.0;
        },
        [&] {
          if (r == r0) {  // the filter block and phases, once for all columns
            mshift_stage(F, Fs, Q, q0);
            for (int e = threadIdx.x; e < 8 * Q; e += blockDim.x) phs[e] = ph[e];
            __syncthreads();
          }
        },
        acc);
    // epilogue from the accumulators: result register v of lane l is
    // D[l / 16 + 4 v][l % 16] of tile (t, ct); columns 2m and 2m + 1 (adjacent
    // lanes) are the real and imaginary parts of one complex value, which the
    // even lane adds to the child's incoming pattern
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        if (!col_ok[ct]) continue;
        const int col = w * 32 + ct * 16 + jl, ci = col / 10, rem = col - ci * 10;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double mine = acc[t][ct][v];
          const double other = __shfl_xor(mine, 1);
          const int i = t * 16 + (lane >> 4) + 4 * v;
          if (!(lane & 1) && valid[ct] && i < nq) {
            cx<double>* o = Gc + (((size_t)(c0 + ci) * R + r) * Q + q0 + i) * 5 + (rem >> 1);
            *o = *o + mk(mine, other);
          }
        }
      }
  }
}

// Downward shift on the matrix cores for batched passes (W >= TB_MIN_COLS).
// A workgroup owns one child c and its output rows q0 .. q0 + 31 and walks
// the MS_COLS blocks of real columns n of a sample row:
//   G_c[q][n] += sum_k F[k][q] (conj(ph_c(k)) G_p[k])[n]
// with the parent's sample rows phased as they are loaded (a lane loads the
// complex value whose real or imaginary part it supplies; 16 lanes cover 128
// consecutive bytes) and the filter block staged once for all column blocks.
__global__ void __launch_bounds__(256, 3) k_mshift_down(DevLevel Lc, const cx<double>* __restrict__ Gp,
                                                     cx<double>* __restrict__ Gc, const double* __restrict__ F,
                                                     const cx<double>* __restrict__ ph, int Q, int R, int ntile) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* Fs = (double*)smem;                                              // filter block
  cx<double>* phs = (cx<double>*)(Fs + mshift_smem(Q) / sizeof(double));   // [Q] phases of the child's octant
  ShiftItem it;
  if (!shift_item(Lc.nb, ntile, 1, MS_ROWS, it)) return;
  const int c = it.g, q0 = it.q0, nq = min(MS_ROWS, Q - q0);
  const int ncol = 10 * R, nnb = (ncol + MS_COLS - 1) / MS_COLS;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, jl = lane & 15;
  const bool im = lane & 1;
  const cx<double>* G = Gp + (size_t)Lc.parent[c] * Q * R * 5;
  double* out = (double*)Gc + ((size_t)c * Q + q0) * ncol;
  mshift_stage(F, Fs, Q, q0);
  for (int e = threadIdx.x; e < Q; e += blockDim.x) phs[e] = ph[(size_t)Lc.octant[c] * Q + e];
  __syncthreads();
  for (int nb = 0; nb < nnb; ++nb) {
    int col[2];
    bool col_ok[2], valid[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int cbase = nb * MS_COLS + w * 32 + ct * 16;
      col_ok[ct] = cbase < ncol;
      valid[ct] = cbase + jl < ncol;
      col[ct] = valid[ct] ? cbase + jl : 0;
    }
    f64x4 acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) acc[t][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
    // the child's current values (result register v of lane l is row
    // l / 16 + 4 v of tile (t, ct)) load after the first operand batch, so
    // that they arrive while the product runs
    double old[2][2][4];
    mshift_gemm<2, cx<double>>(
        Fs, Q, col_ok, [&](int ct, int k) { return G[(size_t)k * R * 5 + (col[ct] >> 1)]; },
        [&](int ct, int k, const cx<double>& g) {
          const cx<double> v = conj(phs[k]) * g;
          return valid[ct] ? (im ? v.im : v.re) : 0.0;
        },
        [&] {
#pragma unroll
          for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                old[t][ct][v] = out[min(t * 16 + (lane >> 4) + 4 * v, nq - 1) * ncol + col[ct]];
        },
        acc);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = t * 16 + (lane >> 4) + 4 * v;
          if (valid[ct] && i < nq) out[i * ncol + col[ct]] = old[t][ct][v] + acc[t][ct][v];
        }
  }
}

// ---------------------------------------------------------------------------
// Translation over the interaction list at one level:
//   G_b(q) = sum_{b' in IL(b)} T_{off(b,b')}(q) S_b'(q)
// a gather (no atomics), for narrow passes (column-major patterns; batched
// passes take k_translate_rows).  One workgroup per (box, RHS column); the list is
// staged in LDS, thread (g, q) takes the entries g (mod nsplit) for all five
// components with four entries' loads in flight, and the nsplit partial
// sums are added in a fixed order through LDS.  nsplit depends on Q only,
// so every RHS column is summed in the same order.
// ---------------------------------------------------------------------------
// (the body takes its box slot bx and column r as arguments so that one
// launch can serve several levels)
template <typename TF>
__device__ __forceinline__ void translate_body(const DevLevel& Lv, const cx<TF>* __restrict__ S,
                                               const cx<TF>* __restrict__ T, cx<TF>* __restrict__ Gout, int Q,
                                               int R, int nsplit, int bx, int r, unsigned char* smem) {
  int32_t* ils = (int32_t*)smem;                 // [IL_MAX + 3]
  int32_t* ilo = ils + (IL_MAX + 3);             // [IL_MAX + 3]
  cx<TF>* part = (cx<TF>*)(ilo + (IL_MAX + 3));  // [nsplit - 1][width][5]
  const int b = xcd_box(bx, Lv.nb);
  if (b < 0) return;
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
      const cx<TF>* Sq = S + ((size_t)r * Q + q) * 5;
      for (int kk = gsp; kk < nil; kk += U * nsplit) {
        cx<TF> tv[U], sv[U][5];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = kk + u * nsplit;
          const bool ok = e < nil;
          tv[u] = ok ? T[(size_t)ilo[e] * Q + q] : mk<TF>(0, 0);
          const cx<TF>* sp = Sq + (size_t)(ok ? ils[e] : 0) * n;
#pragma unroll
          for (int k = 0; k < 5; ++k) sv[u][k] = sp[k];
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
      cx<TF>* o = Gout + (size_t)b * n + ((size_t)r * Q + q) * 5;
#pragma unroll
      for (int k = 0; k < 5; ++k) o[k] = acc[k];
    }
    __syncthreads();
  }
}

template <typename TF>
__global__ void __launch_bounds__(512) k_translate(DevLevel Lv, const cx<TF>* __restrict__ S,
                                                   const cx<TF>* __restrict__ T, cx<TF>* __restrict__ Gout,
                                                   int Q, int R, int nsplit) {
  extern __shared__ __align__(16) unsigned char smem[];
  translate_body<TF>(Lv, S, T, Gout, Q, R, nsplit, blockIdx.x, blockIdx.y, smem);
}

// Several levels' translations in one launch (they are independent once
// the upward pass is done): blocks [off[i], off[i + 1]) serve level i, each
// with the arithmetic of k_translate.
struct TranslateSet {
  int32_t n;
  int32_t off[TSET_MAX + 1];
  DevLevel lv[TSET_MAX];
  const void* S[TSET_MAX];
  const void* T[TSET_MAX];
  void* G[TSET_MAX];
};

template <typename TF>
__global__ void __launch_bounds__(512) k_translate_set(TranslateSet ts, int Q, int R, int nsplit) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int v = blockIdx.x;
  int i = 0;
  while (i + 1 < ts.n && v >= ts.off[i + 1]) ++i;
  const int loc = v - ts.off[i], nx = (int)xcd_grid(ts.lv[i].nb);
  translate_body<TF>(ts.lv[i], (const cx<TF>*)ts.S[i], (const cx<TF>*)ts.T[i], (cx<TF>*)ts.G[i], Q, R, nsplit,
                     loc % nx, loc / nx, smem);
}

// ---------------------------------------------------------------------------
// Reception at the finest level and join with the near-field partial sums.
// Receiving patterns are the conjugates of the radiation patterns, so with
// the moments of each incidence j
//   A = sum_q conj(M1).G_J,  B = sum_q conj(M0) G_J,
//   Cs = sum_q conj(M0) G_sigma,  Du = sum_q conj(M0) G_u,
// an RWG half s (r - p) tests the vector part to mu0 s (A - (p - C).B); at
// its home incidence a triangle receives phi = Cs (the potential of the
// sigma sources) and psi = Du (its pulse row).  Thread (incidence, slice of
// the stored samples) sums its slice, each stored sample s together with
// its antipode (receiving factors conj M(s) and M(s)); the eight slices are
// added by a fixed butterfly.  Each unknown then adds its halves, its
// near-field partial sums in a fixed order (slot lists staged in LDS), and
// is written to its canonical position (conjugated for the adjoint); phi
// goes to a per-triangle array for the divergence testing of the RWG rows.
// ---------------------------------------------------------------------------
// Staged near-field join list of finest box b.  For each of its near boxes
// (chunk c of 128 slots of a structure) the row and then the column
// partial-sum slots are listed, each as (slot - 128 c), so that entry + ul
// addresses the row of the box's unknown ul; kofs[0..nJ] are the list
// ranges of the RWG chunks and kofs[nJ + 1 .. nJ + 1 + nT] those of the
// triangle chunks (the list itself starts at kofs + nJ + nT + 2, returned in
// slots).  Called by every thread of the workgroup (it holds a barrier).
__device__ __forceinline__ void near_join_slots(const DevNear& NJ, const DevNear& NT, int b, bool do_near,
                                                int32_t* kofs, int32_t*& slots, int& nJ) {
  const int vJ0 = NJ.vptr[b], vT0 = NT.vptr[b];
  nJ = NJ.vptr[b + 1] - vJ0;
  const int nT = NT.vptr[b + 1] - vT0;
  slots = kofs + nJ + nT + 2;
  if (threadIdx.x == 0) {
    int k = 0;
    for (int c = 0; c < nJ; ++c) {
      kofs[c] = k;
      const int v = vJ0 + c;
      if (do_near) k += (NJ.row_ptr[v + 1] - NJ.row_ptr[v]) + (NJ.col_ptr[v + 1] - NJ.col_ptr[v]);
    }
    kofs[nJ] = k;
    for (int c = 0; c < nT; ++c) {
      kofs[nJ + 1 + c] = k;
      const int v = vT0 + c;
      if (do_near) k += (NT.row_ptr[v + 1] - NT.row_ptr[v]) + (NT.col_ptr[v + 1] - NT.col_ptr[v]);
    }
    kofs[nJ + 1 + nT] = k;
  }
  __syncthreads();
  const int total = kofs[nJ + 1 + nT], nJs = kofs[nJ];
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c = 0, sl;
    if (e < nJs) {
      while (e >= kofs[c + 1]) ++c;
      const int v = vJ0 + c, f = e - kofs[c], nrow = NJ.row_ptr[v + 1] - NJ.row_ptr[v];
      sl = f < nrow ? NJ.prow[NJ.row_ptr[v] + f] : NJ.pcol[NJ.col_blk[NJ.col_ptr[v] + f - nrow]];
    } else {
      while (e >= kofs[nJ + 2 + c]) ++c;
      const int v = vT0 + c, f = e - kofs[nJ + 1 + c], nrow = NT.row_ptr[v + 1] - NT.row_ptr[v];
      sl = f < nrow ? NT.prow[NT.row_ptr[v] + f] : NT.pcol[NT.col_blk[NT.col_ptr[v] + f - nrow]];
    }
    slots[e] = sl - 128 * c;
  }
}

// Sum of the near partial sums of one unknown: slots [k0, k1) of the staged
// list, local index ul in its structure, column col of a [slot][ld] array.
template <typename TN>
__device__ __forceinline__ void near_join(const cx<TN>* __restrict__ part, const int32_t* slots, int k0, int k1,
                                          int ul, int ld, size_t col, cx<double>& val) {
  int k = k0;
  for (; k + 4 <= k1; k += 4) {
    cx<TN> v[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) v[tt] = part[((size_t)slots[k + tt] + ul) * ld + col];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      val.re += (double)v[tt].re;
      val.im += (double)v[tt].im;
    }
  }
  for (; k < k1; ++k) {
    const cx<TN> v = part[((size_t)slots[k] + ul) * ld + col];
    val.re += (double)v.re;
    val.im += (double)v.im;
  }
}

// Per-unknown assembly of the reception (both reception kernels): an RWG
// row gets its halves' vector testing mu0 s (A - (p - C).B) and the
// RWG-RWG near sums; a triangle (pulse row) gets psi = Du + the S near sums
// of u, which is its output, and phi = Cs + the S near sums of x_A, the
// potential that the RWG rows on the triangle test with their divergence
// (added by k_div_test).  rv(h, o) returns the incidence sum o of half h.
template <typename TN, typename RV>
__device__ __forceinline__ void receive_unknown(const DevInc& I, const DevBasis& B, int u, int ul, int nJb, int r,
                                                int c0, int W, bool do_far, bool do_near, bool conj_out,
                                                const cx<TN>* __restrict__ partJ, const cx<TN>* __restrict__ partT,
                                                const int32_t* slots, const int32_t* kofs, int nJ, RV rv,
                                                cx<double>* __restrict__ y, int ldy, cx<double>* __restrict__ phi) {
  const double mu0 = 4.0e-7 * 3.14159265358979323846;
  const int cu = B.perm[u];
  const size_t col = (size_t)c0 + r;
  if (cu < B.ne) {
    cx<double> val = mk(0.0, 0.0);
    if (do_far) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double sv = I.us[2 * u + h];
        cx<double> t = rv(h, 0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double pc = I.upv[6 * (size_t)u + 3 * h + c];
          const cx<double> bc = rv(h, 1 + c);
          t.re -= pc * bc.re;
          t.im -= pc * bc.im;
        }
        val.re += mu0 * sv * t.re;
        val.im += mu0 * sv * t.im;
      }
    }
    if (do_near) near_join(partJ, slots, kofs[ul >> 7], kofs[(ul >> 7) + 1], ul, W, col, val);
    if (conj_out) val.im = -val.im;
    y[(size_t)cu * ldy + col] = val;
  } else {
    cx<double> ph = mk(0.0, 0.0), ps = mk(0.0, 0.0);
    if (do_far) {
      ph = rv(0, 4);
      ps = rv(0, 5);
    }
    if (do_near) {
      const int lt = ul - nJb, k0 = kofs[nJ + 1 + (lt >> 7)], k1 = kofs[nJ + 2 + (lt >> 7)];
      near_join(partT, slots, k0, k1, lt, 2 * W, col, ph);
      near_join(partT, slots, k0, k1, lt, 2 * W, (size_t)W + col, ps);
    }
    if (conj_out) {
      ph.im = -ph.im;
      ps.im = -ps.im;
    }
    y[(size_t)cu * ldy + col] = ps;
    phi[(size_t)(cu - B.ne) * W + col] = ph;
  }
}

constexpr int RECV_SLICES = 8;  // lanes per incidence (a power of two)
template <typename TF, typename TN, int RC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RC == 1 ? 4 : 1))) k_receive(DevInc I, DevBasis B, DevNear NJ, DevNear NT, int nbox,
                                                 const cx<TF>* __restrict__ Gin, const cx<TF>* __restrict__ M,
                                                 const int32_t* __restrict__ anti, int Q, int Qh,
                                                 const cx<TN>* __restrict__ partJ, const cx<TN>* __restrict__ partT,
                                                 int flags, int W, cx<double>* __restrict__ y, int ldy,
                                                 cx<double>* __restrict__ phi) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_box(blockIdx.x, nbox);
  if (b < 0) return;
  const int j0 = I.ptr[b], ni = I.ptr[b + 1] - j0;
  const PatStride ps = pat_stride(Q, W);
  constexpr int ncol = 5 * RC;
  const bool do_far = flags & 2, do_near = flags & 1, conj_out = flags & 4;
  cx<TF>* Gs = (cx<TF>*)smem;                              // [Q][5][RC]
  cx<TF>* red = Gs + (size_t)Q * ncol;                     // [ni][6][RC]: A, Bx, By, Bz, Cs, Du
  int32_t* pair = (int32_t*)(red + (size_t)ni * 6 * RC);  // [Qh] antipode of each stored sample
  int32_t* kofs = pair + Q;                                // near-field join ranges and slots
  int32_t* slots;
  int nJ;
  near_join_slots(NJ, NT, b, do_near, kofs, slots, nJ);
  if (do_far)
    for (int q = Qh + threadIdx.x; q < Q; q += blockDim.x) pair[anti[q]] = q;
  const int u0 = I.uptr[b], nu = I.uptr[b + 1] - u0;
  const int nJb = NJ.slot_ptr[NJ.vptr[b + 1]] - NJ.slot_ptr[NJ.vptr[b]];  // RWG functions come first in a box
  for (int c0 = 0; c0 < W; c0 += RC) {
    if (c0 > 0) __syncthreads();
    if (do_far) {
      for (int e = threadIdx.x; e < Q * ncol; e += blockDim.x) {
        // source order: that of the layout (sample, column, component when
        // batched; column, sample, component otherwise)
        int q, r, k;
        if (W >= TB_MIN_COLS) {
          q = e / ncol;
          const int rk = e - q * ncol;
          r = rk / 5;
          k = rk - r * 5;
        } else {
          r = e / (5 * Q);
          const int qk = e - r * 5 * Q;
          q = qk / 5;
          k = qk - q * 5;
        }
        Gs[(size_t)q * ncol + k * RC + r] =
            c0 + r < W ? Gin[(size_t)b * Q * W * 5 + (size_t)q * ps.qs + (size_t)(c0 + r) * ps.rs + k]
                       : mk<TF>(0, 0);
      }
    }
    __syncthreads();
    if (do_far) {
      for (int base = 0; base < ni * RECV_SLICES; base += blockDim.x) {
        const int t = base + threadIdx.x;
        const int jl = t / RECV_SLICES, sl = t - jl * RECV_SLICES;
        const bool act = jl < ni;
        cx<TF> acc[6 * RC];
#pragma unroll
        for (int c = 0; c < 6 * RC; ++c) acc[c] = mk<TF>(0, 0);
        if (act) {
          // slice sl takes the stored samples s = sl (mod RECV_SLICES), so the
          // lanes of an incidence read adjacent entries of its moment row.
          // The receiving factor of sample s is conj M(s); that of its
          // antipode pair[s] (when stored samples are halved) is M(s)
          // itself, so every stored moment is loaded once and used twice.
          // Four samples' moments are loaded together before their arithmetic.
          const cx<TF>* mp = M + ((size_t)(j0 + jl) * Qh) * 4;
          auto recv = [&](const cx<TF>(&mm)[4], int q) {
            const cx<TF>* gq = Gs + (size_t)q * ncol;
#pragma unroll
            for (int r = 0; r < RC; ++r) {
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                const cx<TF> gc = gq[c * RC + r];
                cfma(acc[r], mm[1 + c], gc);
                cfma(acc[(1 + c) * RC + r], mm[0], gc);
              }
              cfma(acc[4 * RC + r], mm[0], gq[3 * RC + r]);
              cfma(acc[5 * RC + r], mm[0], gq[4 * RC + r]);
            }
          };
          constexpr int U = 4;
          for (int s0 = sl; s0 < Qh; s0 += U * RECV_SLICES) {
            cx<TF> m[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int su = s0 + u * RECV_SLICES;
              const cx<TF>* ms = mp + 4 * (size_t)(su < Qh ? su : 0);  // in-bounds dummy for the tail
#pragma unroll
              for (int k = 0; k < 4; ++k) m[u][k] = ms[k];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int su = s0 + u * RECV_SLICES;
              if (su < Qh) {
                cx<TF> cm[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) cm[k] = conj(m[u][k]);
                recv(cm, su);
                if (Qh < Q) recv(m[u], pair[su]);
              }
            }
          }
        }
        // fixed butterfly over the RECV_SLICES lanes of an incidence
#pragma unroll
        for (int c = 0; c < 6 * RC; ++c)
#pragma unroll
          for (int h = 1; h < RECV_SLICES; h <<= 1) {
            acc[c].re += __shfl_xor(acc[c].re, h);
            acc[c].im += __shfl_xor(acc[c].im, h);
          }
        if (act && sl == 0) {
#pragma unroll
          for (int c = 0; c < 6 * RC; ++c) red[(size_t)jl * 6 * RC + c] = acc[c];
        }
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < nu * RC; e += blockDim.x) {
      const int ul = e / RC, r = e - ul * RC;
      if (c0 + r >= W) continue;
      const int u = u0 + ul;
      auto rv = [&](int h, int o) {
        const cx<TF> v = red[(size_t)(I.uj[2 * u + h] - j0) * 6 * RC + o * RC + r];
        return mk((double)v.re, (double)v.im);
      };
      receive_unknown<TN>(I, B, u, ul, nJb, r, c0, W, do_far, do_near, conj_out, partJ, partT, slots, kofs,
                          nJ, rv, y, ldy, phi);
    }
  }
}

// ---------------------------------------------------------------------------
// Batched FP64 reception on the matrix cores (W >= MR_COLS columns in a
// pass).  For a box and a block of MR_COLS columns the six sums per
// incidence (A, B, Cs, Du as in k_receive) are complex GEMMs over the stored
// samples s: with M(s) = Mr + i Mi and, per pattern component, the sums
// Sg = G(s) + G(anti s) and Dg = G(s) - G(anti s) of the incoming pattern,
//   conj M(s) G(s) + M(s) G(anti s) = (Mr Sg_r + Mi Dg_i) + i (Mr Sg_i - Mi Dg_r),
// so every moment again serves both samples.  Rows are incidences (row tile
// rt of 16), K steps four stored samples, the (Sg, Dg) of MR_KC samples at
// a time are staged in LDS; with one or two row tiles the waves also split
// the K steps and their partial sums are added through LDS in a fixed
// order.  The per-unknown assembly, the near-field join and the output
// permutation then run as in k_receive.
// ---------------------------------------------------------------------------
constexpr int MR_COLS = 16;
static_assert(MR_COLS >= TB_MIN_COLS, "the matrix-core reception reads sample-major patterns");
constexpr int MR_KC = 16;  // stored samples per staged chunk (four K steps)
constexpr int MR_MAXI = 64;  // incidences per box (four row tiles)

// LDS: one region for the staged (Sg, Dg), then the K-split partial sums,
// then the per-incidence sums; after it the antipode table and the slots.
size_t mreceive_buf(int maxinc) {
  const size_t sd = (size_t)MR_KC * 5 * MR_COLS * 2 * sizeof(cx<double>);
  const size_t pa = (size_t)2 * 64 * 48 * sizeof(double);
  const size_t rd = (size_t)maxinc * 6 * MR_COLS * sizeof(cx<double>);
  return std::max(std::max(sd, pa), rd);
}
size_t mreceive_smem(int maxinc, int maxjoin, int Q) {
  return mreceive_buf(maxinc) + (size_t)(maxjoin + Q) * sizeof(int32_t) + 16;
}

template <typename TN>
__global__ void __launch_bounds__(256) k_mreceive(DevInc I, DevBasis B, DevNear NJ, DevNear NT, int nbox,
                                                  const cx<double>* __restrict__ Gin, const cx<double>* __restrict__ M,
                                                  const int32_t* __restrict__ anti, int Q, int Qh, size_t buf,
                                                  const cx<TN>* __restrict__ partJ, const cx<TN>* __restrict__ partT,
                                                  int flags, int W, cx<double>* __restrict__ y, int ldy,
                                                  cx<double>* __restrict__ phi) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_box(blockIdx.x, nbox);
  if (b < 0) return;
  const int c0 = blockIdx.y * MR_COLS;
  const int j0 = I.ptr[b], ni = I.ptr[b + 1] - j0;
  const bool do_far = flags & 2, do_near = flags & 1, conj_out = flags & 4;
  cx<double>* SD = (cx<double>*)smem;    // [MR_KC][5][MR_COLS][2]: Sg, Dg
  double* pa = (double*)smem;            // [2][64][48] partial sums of the K split
  cx<double>* red = (cx<double>*)smem;   // [ni][6][MR_COLS]
  int32_t* pairt = (int32_t*)(smem + buf);  // [Q] antipode of each stored sample
  int32_t* kofs = pairt + Q;                  // near-field join ranges and slots
  int32_t* slots;
  int nJ;
  near_join_slots(NJ, NT, b, do_near, kofs, slots, nJ);
  const bool paired = Qh < Q;
  for (int q = Qh + threadIdx.x; q < Q; q += blockDim.x) pairt[anti[q]] = q;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, kq = lane >> 4, jl = lane & 15;
  const int nrt = (ni + 15) >> 4;  // <= MR_MAXI / 16 (host)
  const int ksplit = nrt == 1 ? 4 : (nrt == 2 ? 2 : 1);
  const int rt = nrt > 0 ? w % nrt : 0, kh = nrt > 0 ? w / nrt : 4;
  const bool wact = do_far && nrt > 0 && kh < ksplit;
  const int jrow = rt * 16 + jl;
  f64x4 acc[6][2];
#pragma unroll
  for (int o = 0; o < 6; ++o) acc[o][0] = acc[o][1] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (do_far) {
    for (int sc = 0; sc < Qh; sc += MR_KC) {
      __syncthreads();  // previous chunk consumed (and pair table / slots written)
      for (int e = threadIdx.x; e < MR_KC * 5 * MR_COLS; e += blockDim.x) {
        // source order: sample, column, component (one contiguous run per sample)
        const int si = e / (5 * MR_COLS), rem = e - si * (5 * MR_COLS), r = rem / 5, k = rem - r * 5;
        const int sv = sc + si;
        cx<double> a = mk(0.0, 0.0), c = mk(0.0, 0.0);
        if (sv < Qh && c0 + r < W) {
          const cx<double>* g = Gin + ((size_t)b * Q * W + c0 + r) * 5 + k;
          a = g[(size_t)sv * W * 5];
          if (paired) c = g[(size_t)pairt[sv] * W * 5];
        }
        SD[((si * 5 + k) * MR_COLS + r) * 2] = a + c;
        SD[((si * 5 + k) * MR_COLS + r) * 2 + 1] = a - c;
      }
      __syncthreads();
      if (wact) {
#pragma unroll
        for (int t = 0; t < MR_KC / 4; ++t) {
          if (t % ksplit != kh) continue;
          const int si = 4 * t + kq, sv = sc + si;
          const bool ok = sv < Qh && jrow < ni;
          const cx<double>* mp = M + ((size_t)(j0 + (ok ? jrow : 0)) * Qh + (ok ? sv : 0)) * 4;
          cx<double> m[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const cx<double> v = mp[u];
            m[u] = ok ? v : mk(0.0, 0.0);
          }
          // (moment, component) -> output: M1c.G_Jc -> A; M0.G_Jc -> Bc; M0.G_sigma -> Cs; M0.G_u -> Du
#pragma unroll
          for (int pi = 0; pi < 8; ++pi) {
            const int mi = pi < 3 ? 1 + pi : 0, k = pi < 3 ? pi : pi - 3, o = pi < 3 ? 0 : pi - 2;
            const cx<double> sg = SD[((si * 5 + k) * MR_COLS + jl) * 2];
            const cx<double> dg = SD[((si * 5 + k) * MR_COLS + jl) * 2 + 1];
            acc[o][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(m[mi].re, sg.re, acc[o][0], 0, 0, 0);
            acc[o][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(m[mi].im, dg.im, acc[o][0], 0, 0, 0);
            acc[o][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(m[mi].re, sg.im, acc[o][1], 0, 0, 0);
            acc[o][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(m[mi].im, -dg.re, acc[o][1], 0, 0, 0);
          }
        }
      }
    }
    // K-split partial sums, added to the kh = 0 waves in order of kh
    for (int h = 1; h < ksplit; ++h) {
      __syncthreads();
      if (wact && kh == h) {
        double* pp = pa + ((size_t)rt * 64 + lane) * 48;
#pragma unroll
        for (int o = 0; o < 6; ++o)
#pragma unroll
          for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) pp[(o * 2 + c) * 4 + v] = acc[o][c][v];
      }
      __syncthreads();
      if (wact && kh == 0) {
        const double* pp = pa + ((size_t)rt * 64 + lane) * 48;
#pragma unroll
        for (int o = 0; o < 6; ++o)
#pragma unroll
          for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[o][c][v] += pp[(o * 2 + c) * 4 + v];
      }
    }
    __syncthreads();
    if (wact && kh == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jr = rt * 16 + kq + 4 * v;
        if (jr < ni)
#pragma unroll
          for (int o = 0; o < 6; ++o) red[((size_t)jr * 6 + o) * MR_COLS + jl] = mk(acc[o][0][v], acc[o][1][v]);
      }
    }
  }
  __syncthreads();
  const int u0 = I.uptr[b], nu = I.uptr[b + 1] - u0;
  const int nJb = NJ.slot_ptr[NJ.vptr[b + 1]] - NJ.slot_ptr[NJ.vptr[b]];
  for (int e = threadIdx.x; e < nu * MR_COLS; e += blockDim.x) {
    const int ul = e / MR_COLS, r = e - ul * MR_COLS;
    if (c0 + r >= W) continue;
    const int u = u0 + ul;
    auto rv = [&](int h, int o) { return red[((size_t)(I.uj[2 * u + h] - j0) * 6 + o) * MR_COLS + r]; };
    receive_unknown<TN>(I, B, u, ul, nJb, r, c0, W, do_far, do_near, conj_out, partJ, partT, slots, kofs, nJ,
                        rv, y, ldy, phi);
  }
}

// Canonical FP64 x -> the near-field inputs in near-field precision
// (conjugated for the adjoint): xJ[sJ][W] = x of the RWG function at RWG
// slot sJ; xT[sT][2W] = (x_A, u) of the triangle at triangle slot sT, with
// u = div J + w^2 eps0 x_A formed in FP64 from all the RWG functions on it.
template <typename TN>
__global__ void k_near_in(const cx<double>* __restrict__ x, int ldx, const int32_t* __restrict__ permJ,
                          const int32_t* __restrict__ permT, DevTriDiv td, double w2e, int W, int conjx,
                          cx<TN>* __restrict__ xJ, cx<TN>* __restrict__ xT) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nJ = (int64_t)td.ne * W;
  if (e < nJ) {
    const int sj = (int)(e / W), r = (int)(e - (int64_t)sj * W);
    cx<double> v = x[(size_t)permJ[sj] * ldx + r];
    if (conjx) v.im = -v.im;
    xJ[e] = mk((TN)v.re, (TN)v.im);
    return;
  }
  const int64_t f = e - nJ;
  if (f >= (int64_t)td.nt * W) return;
  const int st = (int)(f / W), r = (int)(f - (int64_t)st * W);
  const int t = permT[st];
  cx<double> xa = x[(size_t)(td.ne + t) * ldx + r];
  if (conjx) xa.im = -xa.im;
  const cx<double> u = tri_u(td, x, ldx, r, t, xa, w2e, conjx);
  xT[(size_t)st * 2 * W + r] = mk((TN)xa.re, (TN)xa.im);
  xT[(size_t)st * 2 * W + W + r] = mk((TN)u.re, (TN)u.im);
}

// RWG rows += G phi: each RWG function tests the per-triangle potential phi
// [T][W] of its two triangles with its divergence +-l/A (the JA block
// G S of the operator; phi already conjugated for the adjoint).  cs holds
// +-l/(2A) per (edge, half), so the divergence is 2 cs exactly.
__global__ void k_div_test(const int32_t* __restrict__ tri, const double* __restrict__ cs,
                           const cx<double>* __restrict__ phi, int ne, int W, cx<double>* __restrict__ y, int ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ne * W) return;
  const int m = (int)(e / W), r = (int)(e - (int64_t)m * W);
  const cx<double> p0 = phi[(size_t)tri[2 * m] * W + r], p1 = phi[(size_t)tri[2 * m + 1] * W + r];
  const double d0 = 2.0 * cs[2 * m], d1 = 2.0 * cs[2 * m + 1];
  cx<double>& o = y[(size_t)m * ldy + r];
  o.re += d0 * p0.re + d1 * p1.re;
  o.im += d0 * p0.im + d1 * p1.im;
}

// ------------------------------------------------------------- launchers --
size_t aggregate_smem(int maxinc, int Q, int nsplit, int RC, int tf_bytes) {
  return (size_t)maxinc * 6 * RC * 2 * tf_bytes + (size_t)(nsplit - 1) * Q * 5 * RC * 2 * tf_bytes +
         (size_t)Q * 4 + 16;
}
size_t receive_smem(int maxinc, int Q, int maxjoin, int RC, int tf_bytes) {
  return (size_t)Q * 5 * RC * 2 * tf_bytes + (size_t)maxinc * 6 * RC * 2 * tf_bytes + (size_t)(Q + maxjoin) * 4 +
         16;
}

template <typename TF>
hipError_t launch_moments(const double* pw, int ninc, const double* khat64, int Qh, double kappa, void* M,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_moments<TF>, dim3(ninc), dim3(128), 0, st, pw, khat64, Qh, kappa, (cx<TF>*)M);
  return hipGetLastError();
}

// W columns per pass (x: [N][ldx] canonical, S: [box][Q][5][W]); rc: widest
// register group (1, 2 or 4).
template <typename TF>
hipError_t launch_aggregate(const DevInc& I, int nb, int maxinc, const void* x, int ldx, int W, int rc,
                            const void* M, const int32_t* anti, int Q, int Qh, double w2e, int conjx, int nsplit,
                            void* S, hipStream_t st) {
  if (W < 1 || (rc != 1 && rc != 2 && rc != 4)) return hipErrorInvalidValue;
  if (nsplit * Qh > 256) return hipErrorInvalidValue;
  if (sizeof(TF) == 8 && W >= MA_COLS && Q <= 256) {
    hipLaunchKernelGGL(k_maggregate, dim3(xcd_grid(nb), (W + MA_COLS - 1) / MA_COLS), dim3(256), 0, st, I, nb,
                       (const cx<double>*)x, ldx, (const cx<double>*)M, anti, Q, Qh, w2e, conjx, W,
                       (cx<double>*)S);
    return hipGetLastError();
  }
  const int g = W >= 4 && rc >= 4 ? 4 : (W >= 2 && rc >= 2 ? 2 : 1);
#define AGG(RC_)                                                                                               \
  hipLaunchKernelGGL((k_aggregate<TF, RC_>), dim3(xcd_grid(nb)), dim3(256),                                    \
                     aggregate_smem(maxinc, Q, nsplit, RC_, sizeof(TF)), st, I, nb, (const cx<double>*)x, ldx, \
                     (const cx<TF>*)M, anti, Q, Qh, w2e, conjx, nsplit, W, (cx<TF>*)S)
  if (g == 1) AGG(1); else if (g == 2) AGG(2); else AGG(4);
#undef AGG
  return hipGetLastError();
}

size_t shift_smem(int Q, int tf_bytes) {
  return (size_t)SHIFT_SLICES * SHIFT_LANES * SQT * 2 * tf_bytes + (size_t)Q * SQT * tf_bytes;
}

template <typename TF>
hipError_t launch_shift_up(const DevLevel& Lp, const DevLevel& Lc, const void* Sc, void* Sp, const void* Ft,
                           const void* ph, int Q, int R, bool force_mfma, hipStream_t st) {
  static_assert(SHIFT_GROUP * 5 <= SHIFT_LANES, "shift group exceeds its lanes");
  // matrix cores when the level has enough (group, row block) items to fill
  // the device, counting 16 columns for batched passes (so that the choice
  // is the same for every batched pass width); the vector kernel (more,
  // shorter work items) otherwise
  if (sizeof(TF) == 8 &&
      (force_mfma || Lp.nug * ((Q + MS_ROWS - 1) / MS_ROWS) * (R >= 16 ? 16 : 1) >= MS_MIN_ITEMS)) {
    const int ntile = (Q + MS_ROWS - 1) / MS_ROWS;
    if (R >= TB_MIN_COLS) {
      const int nnb = (10 * R + MS_COLS - 1) / MS_COLS;
      const unsigned grid = 8u * (unsigned)(((Lp.nb + 7) / 8) * ntile * nnb);
      const size_t sm = mshift_smem(Q) + 8 * MS_ROWS * sizeof(cx<double>);
      hipLaunchKernelGGL(k_mshift_up, dim3(grid), dim3(256), sm, st, Lp, Lc, (const cx<double>*)Sc,
                         (cx<double>*)Sp, (const double*)Ft, (const cx<double>*)ph, Q, R, ntile, nnb);
      return hipGetLastError();
    }
    const int nchunk = (R + MS_RCH - 1) / MS_RCH;
    const unsigned grid = 8u * (unsigned)(((Lp.nug + 7) / 8) * ntile * nchunk);
    const size_t sm = MS_ROWS * MS_COLS * sizeof(double) + SHIFT_GROUP * MS_ROWS * sizeof(cx<double>) +
                      (SHIFT_GROUP + 1) * sizeof(int32_t);
    hipLaunchKernelGGL(k_mshift_up_groups, dim3(grid), dim3(256), sm, st, Lp, Lc, (const cx<double>*)Sc,
                       (cx<double>*)Sp, (const double*)Ft, (const cx<double>*)ph, Q, R, ntile, nchunk);
    return hipGetLastError();
  }
  const int ntile = (Q + SQT - 1) / SQT;
  const unsigned grid = 8u * (unsigned)(((Lp.nug + 7) / 8) * ntile * R);
  hipLaunchKernelGGL(k_shift_up<TF>, dim3(grid), dim3(SHIFT_SLICES * SHIFT_LANES), shift_smem(Q, sizeof(TF)), st,
                     Lp, Lc, (const cx<TF>*)Sc, (cx<TF>*)Sp, (const TF*)Ft, (const cx<TF>*)ph, Q, R, ntile);
  return hipGetLastError();
}

template <typename TF>
hipError_t launch_shift_down(const DevLevel& Lc, const void* Gp, void* Gc, const void* F, const void* ph, int Q,
                             int R, bool force_mfma, hipStream_t st) {
  const int ng = (Lc.nb + SHIFT_GROUP - 1) / SHIFT_GROUP;
  if (sizeof(TF) == 8 && (force_mfma || ng * ((Q + MS_ROWS - 1) / MS_ROWS) * (R >= 16 ? 16 : 1) >= MS_MIN_ITEMS)) {
    const int ntile = (Q + MS_ROWS - 1) / MS_ROWS;
    if (R >= TB_MIN_COLS) {
      const unsigned grid = 8u * (unsigned)(((Lc.nb + 7) / 8) * ntile);
      const size_t sm = mshift_smem(Q) + (size_t)Q * sizeof(cx<double>);
      hipLaunchKernelGGL(k_mshift_down, dim3(grid), dim3(256), sm, st, Lc, (const cx<double>*)Gp,
                         (cx<double>*)Gc, (const double*)F, (const cx<double>*)ph, Q, R, ntile);
      return hipGetLastError();
    }
    const int nchunk = (R + MS_RCH - 1) / MS_RCH;
    const unsigned grid = 8u * (unsigned)(((ng + 7) / 8) * ntile * nchunk);
    const size_t sm = mshift_smem(Q) + 8 * (size_t)Q * sizeof(cx<double>);
    hipLaunchKernelGGL(k_mshift_down_groups, dim3(grid), dim3(256), sm, st, Lc, (const cx<double>*)Gp, (cx<double>*)Gc,
                       (const double*)F, (const cx<double>*)ph, Q, R, ntile, nchunk);
    return hipGetLastError();
  }
  const int ntile = (Q + SQT - 1) / SQT;
  const unsigned grid = 8u * (unsigned)(((ng + 7) / 8) * ntile * R);
  hipLaunchKernelGGL(k_shift_down<TF>, dim3(grid), dim3(SHIFT_SLICES * SHIFT_LANES), shift_smem(Q, sizeof(TF)),
                     st, Lc, (const cx<TF>*)Gp, (cx<TF>*)Gc, (const TF*)F, (const cx<TF>*)ph, Q, R, ntile);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched translation (W >= TB_MIN_COLS columns in a pass).  For one sample q
// the translation of Eq. (4) scales whole pattern rows: the W x 5 values
// S[box][q][r][c] of every source in a box's list are multiplied by the one
// factor T[off][q] and summed.  A wavefront owns (translation group, q, a
// chunk of <= TG_COLS columns): its lanes hold the chunk's (r, c) values
// (NS per lane; one load instruction covers 64 consecutive values of the
// sample-major row), so the factor is wavefront-uniform (scalar loads) and
// each source row loaded into registers is used for every box of the group
// that lists it (the group's union is walked once, in ascending source
// order, which is also each box's summation order).  Workgroup = TG_Q
// samples of one group; chunk slowest, then the sample block, then the
// group: each XCD takes whole sample blocks and walks the groups in Morton
// order, so the workgroups resident on it at one time share their source
// rows in its L2.
// ---------------------------------------------------------------------------

template <typename TF, int NS>
__global__ void __launch_bounds__(64 * TG_Q) k_translate_rows(DevLevel Lv, const cx<TF>* __restrict__ S,
                                                        const cx<TF>* __restrict__ T, cx<TF>* __restrict__ Gout,
                                                        int Q, int W, int nqb, int cols) {
  const int it = xcd_box(blockIdx.x, Lv.ntg * nqb * ((W + cols - 1) / cols));
  if (it < 0) return;
  const int g = it % Lv.ntg, rest = it / Lv.ntg;
  const int qb = rest % nqb, chunk = rest / nqb;
  const int q = qb * TG_Q + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (q >= Q) return;
  const int lane = threadIdx.x & 63;
  const int c0 = chunk * cols, nv = 5 * min(cols, W - c0);
  // value offsets in a pattern row (-1: no value); load offsets (always in the row)
  int off[NS], ld[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int e = i * 64 + lane;
    off[i] = e < nv ? (q * W + c0) * 5 + e : -1;
    ld[i] = off[i] < 0 ? 0 : off[i];
  }
  const size_t row = (size_t)W * Q * 5;
  const int b0 = Lv.tg_box[g], nbx = Lv.tg_box[g + 1] - b0;
  const int j0 = Lv.tg_ent[g], j1 = Lv.tg_ent[g + 1];
  cx<TF> acc[TG_BOXES][NS];
#pragma unroll
  for (int d = 0; d < TG_BOXES; ++d)
#pragma unroll
    for (int i = 0; i < NS; ++i) acc[d][i] = mk<TF>(0, 0);
  // entry j: its source row (lane values) and the factors of its boxes
  // (offset 0xffff: not in that box's list; its factor load reads offset 0)
  auto fetch = [&](int j, int4& en, cx<TF>* v, cx<TF>* t) {
    en = Lv.te[j];
    const cx<TF>* src = S + (size_t)en.x * row;
#pragma unroll
    for (int i = 0; i < NS; ++i) v[i] = src[ld[i]];
#pragma unroll
    for (int d = 0; d < TG_BOXES; ++d) {
      const uint32_t w = (uint32_t)(d < 2 ? en.y : en.z), o = d & 1 ? w >> 16 : w & 0xffffu;
      t[d] = T[(size_t)(o == 0xffffu ? 0u : o) * Q + q];
    }
  };
  auto use = [&](const int4& en, const cx<TF>* v, const cx<TF>* t) {
#pragma unroll
    for (int d = 0; d < TG_BOXES; ++d) {
      const uint32_t w = (uint32_t)(d < 2 ? en.y : en.z), o = d & 1 ? w >> 16 : w & 0xffffu;
      if (o != 0xffffu)
#pragma unroll
        for (int i = 0; i < NS; ++i) cfma(acc[d][i], t[d], v[i]);
    }
  };
  if (j0 < j1) {
    // three register sets: the next two entries' loads are in flight while
    // the current one is summed (prefetches past the end re-read the last)
    int4 eA, eB, eC;
    cx<TF> sA[NS], sB[NS], sC[NS], tA[TG_BOXES], tB[TG_BOXES], tC[TG_BOXES];
    fetch(j0, eA, sA, tA);
    fetch(min(j0 + 1, j1 - 1), eB, sB, tB);
    for (int j = j0;;) {
      fetch(min(j + 2, j1 - 1), eC, sC, tC);
      use(eA, sA, tA);
      if (++j >= j1) break;
      fetch(min(j + 2, j1 - 1), eA, sA, tA);
      use(eB, sB, tB);
      if (++j >= j1) break;
      fetch(min(j + 2, j1 - 1), eB, sB, tB);
      use(eC, sC, tC);
      if (++j >= j1) break;
    }
  }
#pragma unroll
  for (int d = 0; d < TG_BOXES; ++d)
    if (d < nbx) {
      cx<TF>* o = Gout + (size_t)(b0 + d) * row;
#pragma unroll
      for (int i = 0; i < NS; ++i)
        if (off[i] >= 0) o[off[i]] = acc[d][i];
    }
}

// Interaction-list split: Q lanes rounded to wavefronts (at most 256 per
// pass) times nsplit list slices in a block of at most 512 threads.
int translate_width(int Q) { return std::min(256, 64 * ((Q + 63) / 64)); }
int translate_split(int Q) { return std::min(8, 512 / translate_width(Q)); }

// Translations of n levels in one launch where every level takes the
// single-column kernel (a batched pass, or more than TSET_MAX levels, uses
// one launch per level); results equal the per-level launches bit for bit.
template <typename TF>
hipError_t launch_translate_levels(const DevLevel* lv, const void* const* S, const void* const* T, void* const* G,
                                   int n, int Q, int R, hipStream_t st) {
  const int width = translate_width(Q), ns = translate_split(Q);
  bool single = n <= TSET_MAX;
  if (R >= TB_MIN_COLS) single = false;
  if (!single) {
    for (int i = 0; i < n; ++i) {
      hipError_t e = launch_translate<TF>(lv[i], S[i], T[i], G[i], Q, R, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (n == 0) return hipSuccess;
  TranslateSet ts{};
  ts.n = n;
  ts.off[0] = 0;
  for (int i = 0; i < n; ++i) {
    ts.lv[i] = lv[i];
    ts.S[i] = S[i];
    ts.T[i] = T[i];
    ts.G[i] = G[i];
    ts.off[i + 1] = ts.off[i] + (int)xcd_grid(lv[i].nb) * R;
  }
  const size_t sm = 2 * (IL_MAX + 3) * sizeof(int32_t) + (size_t)(ns - 1) * width * 5 * 2 * sizeof(TF) + 16;
  hipLaunchKernelGGL(k_translate_set<TF>, dim3(ts.off[n]), dim3(width * ns), sm, st, ts, Q, R, ns);
  return hipGetLastError();
}

template <typename TF>
hipError_t launch_translate(const DevLevel& Lv, const void* S, const void* T, void* Gout, int Q, int R,
                            hipStream_t st) {
  if (R >= TB_MIN_COLS) {
    const int cols = TG_COLS;
    const int nqb = (Q + TG_Q - 1) / TG_Q, nch = (R + cols - 1) / cols;
    const int ns = (5 * std::min(R, cols) + 63) / 64;  // values per lane
    const dim3 grid(xcd_grid(Lv.ntg * nqb * nch));
#define TROWS(NS_)                                                                                               \
  hipLaunchKernelGGL((k_translate_rows<TF, NS_>), grid, dim3(64 * TG_Q), 0, st, Lv, (const cx<TF>*)S,          \
                     (const cx<TF>*)T, (cx<TF>*)Gout, Q, R, nqb, cols)
    if (ns <= 2) TROWS(2); else if (ns == 3) TROWS(3); else if (ns == 4) TROWS(4); else TROWS(5);
#undef TROWS
    return hipGetLastError();
  }
  const int width = translate_width(Q), ns = translate_split(Q);
  const size_t sm = 2 * (IL_MAX + 3) * sizeof(int32_t) + (size_t)(ns - 1) * width * 5 * 2 * sizeof(TF) + 16;
  hipLaunchKernelGGL(k_translate<TF>, dim3(xcd_grid(Lv.nb), R), dim3(width * ns), sm, st, Lv, (const cx<TF>*)S,
                     (const cx<TF>*)T, (cx<TF>*)Gout, Q, R, ns);
  return hipGetLastError();
}

template <typename TF, typename TN>
hipError_t launch_receive(const DevInc& I, const DevBasis& B, const DevNear& NJ, const DevNear& NT, int nb,
                          int maxinc, int maxjoin, const void* Gin, const void* M, const int32_t* anti, int Q, int Qh,
                          const void* partJ, const void* partT, int W, int rc, int flags, void* y, int ldy,
                          void* phi, hipStream_t st) {
  if (W < 1 || (rc != 1 && rc != 2 && rc != 4)) return hipErrorInvalidValue;
  if (sizeof(TF) == 8 && W >= MR_COLS && maxinc <= MR_MAXI) {
    const size_t buf = mreceive_buf(maxinc);
    hipLaunchKernelGGL(k_mreceive<TN>, dim3(xcd_grid(nb), (W + MR_COLS - 1) / MR_COLS), dim3(256),
                       mreceive_smem(maxinc, maxjoin, Q), st, I, B, NJ, NT, nb, (const cx<double>*)Gin,
                       (const cx<double>*)M, anti, Q, Qh, buf, (const cx<TN>*)partJ, (const cx<TN>*)partT, flags,
                       W, (cx<double>*)y, ldy, (cx<double>*)phi);
    return hipGetLastError();
  }
  const int g = W >= 4 && rc >= 4 ? 4 : (W >= 2 && rc >= 2 ? 2 : 1);
#define REC(RC_)                                                                                              \
  hipLaunchKernelGGL((k_receive<TF, TN, RC_>), dim3(xcd_grid(nb)), dim3(256),                                 \
                     receive_smem(maxinc, Q, maxjoin, RC_, sizeof(TF)), st, I, B, NJ, NT, nb, (const cx<TF>*)Gin, \
                     (const cx<TF>*)M, anti, Q, Qh, (const cx<TN>*)partJ, (const cx<TN>*)partT, flags, W,       \
                     (cx<double>*)y, ldy, (cx<double>*)phi)
  if (g == 1) REC(1); else if (g == 2) REC(2); else REC(4);
#undef REC
  return hipGetLastError();
}

template <typename TN>
hipError_t launch_near_in(const void* x, int ldx, const int32_t* permJ, const int32_t* permT, const DevTriDiv& td,
                          double w2e, int W, int conjx, void* xJ, void* xT, hipStream_t st) {
  const int64_t n = ((int64_t)td.ne + td.nt) * W;
  hipLaunchKernelGGL(k_near_in<TN>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const cx<double>*)x, ldx,
                     permJ, permT, td, w2e, W, conjx, (cx<TN>*)xJ, (cx<TN>*)xT);
  return hipGetLastError();
}

hipError_t launch_div_test(const int32_t* tri, const double* cs, const void* phi, int ne, int W, void* y, int ldy,
                           hipStream_t st) {
  const int64_t n = (int64_t)ne * W;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_div_test, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tri, cs,
                     (const cx<double>*)phi, ne, W, (cx<double>*)y, ldy);
  return hipGetLastError();
}

#define INST_F(TF)                                                                                            \
  template hipError_t launch_moments<TF>(const double*, int, const double*, int, double, void*, hipStream_t); \
  template hipError_t launch_aggregate<TF>(const DevInc&, int, int, const void*, int, int, int, const void*,   \
                                           const int32_t*, int, int, double, int, int, void*, hipStream_t); \
  template hipError_t launch_shift_up<TF>(const DevLevel&, const DevLevel&, const void*, void*, const void*,  \
                                          const void*, int, int, bool, hipStream_t);                         \
  template hipError_t launch_shift_down<TF>(const DevLevel&, const void*, void*, const void*, const void*,   \
                                            int, int, bool, hipStream_t);                                    \
  template hipError_t launch_translate_levels<TF>(const DevLevel*, const void* const*, const void* const*,       \
                                                 void* const*, int, int, int, hipStream_t);                    \
  template hipError_t launch_translate<TF>(const DevLevel&, const void*, const void*, void*, int, int,       \
                                           hipStream_t);                                                     \
  template hipError_t launch_near_in<TF>(const void*, int, const int32_t*, const int32_t*, const DevTriDiv&,  \
                                         double, int, int, void*, void*, hipStream_t);
INST_F(float)
INST_F(double)
template hipError_t launch_receive<float, float>(const DevInc&, const DevBasis&, const DevNear&, const DevNear&, int, int, int, const void*, const void*, const int32_t*, int, int, const void*, const void*, int, int, int, void*, int, void*, hipStream_t);
template hipError_t launch_receive<double, float>(const DevInc&, const DevBasis&, const DevNear&, const DevNear&, int, int, int, const void*, const void*, const int32_t*, int, int, const void*, const void*, int, int, int, void*, int, void*, hipStream_t);
template hipError_t launch_receive<float, double>(const DevInc&, const DevBasis&, const DevNear&, const DevNear&, int, int, int, const void*, const void*, const int32_t*, int, int, const void*, const void*, int, int, int, void*, int, void*, hipStream_t);
template hipError_t launch_receive<double, double>(const DevInc&, const DevBasis&, const DevNear&, const DevNear&, int, int, int, const void*, const void*, const int32_t*, int, int, const void*, const void*, int, int, int, void*, int, void*, hipStream_t);

}  // namespace pie
