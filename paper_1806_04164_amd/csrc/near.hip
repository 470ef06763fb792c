// Near-field interactions (Section 3: direct MoM entries of Eqs. (1)-(2) for
// basis functions in one-box-buffer neighbour boxes): fill and SpMM.
#include "device.h"
#include "kernels.h"

namespace pie {

// ---------------------------------------------------------------------------
// Fill: FP64 triangle-pair moments with the 7-point rule on both triangles;
// for pairs that share a vertex, the static part 1/(4 pi R) of the inner
// integral is done in closed form and the pair is averaged with its swap.
// ---------------------------------------------------------------------------
struct Mom {
  cx<double> M0, Mo[3], Ms[3], Mos;
};

// int_T 1/|r-r'| and int_T (r' - rho)/|r-r'| over the triangle (a,b,c)
// (rho = projection of r on its plane), summed edge by edge.
__device__ void tri_potential(const double r[3], const double* va, const double* vb,
                              const double* vc, const double nrm[3], double& K0, double K1[3]) {
  const double d = nrm[0] * (r[0] - va[0]) + nrm[1] * (r[1] - va[1]) + nrm[2] * (r[2] - va[2]);
  const double ad = fabs(d);
  const double rho[3] = {r[0] - d * nrm[0], r[1] - d * nrm[1], r[2] - d * nrm[2]};
  K0 = 0.0;
  K1[0] = K1[1] = K1[2] = 0.0;
  const double* vs[4] = {va, vb, vc, va};
  for (int e = 0; e < 3; ++e) {
    const double* a = vs[e];
    const double* b = vs[e + 1];
    double ed[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double el = sqrt(ed[0] * ed[0] + ed[1] * ed[1] + ed[2] * ed[2]);
    double lh[3] = {ed[0] / el, ed[1] / el, ed[2] / el};
    // in-plane outward edge normal u = lhat x n
    double uh[3] = {lh[1] * nrm[2] - lh[2] * nrm[1], lh[2] * nrm[0] - lh[0] * nrm[2],
                    lh[0] * nrm[1] - lh[1] * nrm[0]};
    double am[3] = {a[0] - rho[0], a[1] - rho[1], a[2] - rho[2]};
    double bm[3] = {b[0] - rho[0], b[1] - rho[1], b[2] - rho[2]};
    double t = am[0] * uh[0] + am[1] * uh[1] + am[2] * uh[2];
    double sm = am[0] * lh[0] + am[1] * lh[1] + am[2] * lh[2];
    double sp = bm[0] * lh[0] + bm[1] * lh[1] + bm[2] * lh[2];
    double ra[3] = {r[0] - a[0], r[1] - a[1], r[2] - a[2]};
    double rb[3] = {r[0] - b[0], r[1] - b[1], r[2] - b[2]};
    double Rm = sqrt(ra[0] * ra[0] + ra[1] * ra[1] + ra[2] * ra[2]);
    double Rp = sqrt(rb[0] * rb[0] + rb[1] * rb[1] + rb[2] * rb[2]);
    double R0sq = t * t + d * d;
    // R + s computed as R0^2/(R - s) when s < 0 (no cancellation)
    double num = sp >= 0.0 ? Rp + sp : (Rp - sp > 0.0 ? R0sq / (Rp - sp) : 0.0);
    double den = sm >= 0.0 ? Rm + sm : (Rm - sm > 0.0 ? R0sq / (Rm - sm) : 0.0);
    double f = (num > 0.0 && den > 0.0) ? log(num / den) : 0.0;
    double beta = atan2(t * sp, R0sq + ad * Rp) - atan2(t * sm, R0sq + ad * Rm);
    K0 += t * f - ad * beta;
    double g = 0.5 * (R0sq * f + sp * Rp - sm * Rm);
    K1[0] += g * uh[0];
    K1[1] += g * uh[1];
    K1[2] += g * uh[2];
  }
}

__device__ void raw_moments(const DevGeo& G, int ta, int tb, bool touch, double k, Mom& m) {
  const double* Pa = G.P + 21 * ta;
  const double* Pb = G.P + 21 * tb;
  const double* Wa = G.W + 7 * ta;
  const double* Wb = G.W + 7 * tb;
  const double* ca = G.C + 3 * ta;
  const double* cb = G.C + 3 * tb;
  const double inv4pi = 0.25 / 3.14159265358979323846;
  m.M0 = mk(0.0, 0.0);
  m.Mos = mk(0.0, 0.0);
  for (int d = 0; d < 3; ++d) m.Mo[d] = m.Ms[d] = mk(0.0, 0.0);
  for (int i = 0; i < 7; ++i) {
    double ra[3] = {Pa[3 * i] - ca[0], Pa[3 * i + 1] - ca[1], Pa[3 * i + 2] - ca[2]};
    cx<double> gi = mk(0.0, 0.0);
    cx<double> hi[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    for (int j = 0; j < 7; ++j) {
      double dx = Pa[3 * i] - Pb[3 * j], dy = Pa[3 * i + 1] - Pb[3 * j + 1], dz = Pa[3 * i + 2] - Pb[3 * j + 2];
      double R = sqrt(dx * dx + dy * dy + dz * dz);
      cx<double> g;
      if (!touch) {
        double sn, cs;
        sincos(k * R, &sn, &cs);
        double f = inv4pi / R;
        g = mk(cs * f, sn * f);
      } else {
        // (exp(ikR) - 1)/(4 pi R) = (ik/4pi) exp(ikR/2) sin(kR/2)/(kR/2)
        double h = 0.5 * k * R;
        double sinc = fabs(h) < 1e-4 ? 1.0 - h * h / 6.0 : sin(h) / h;
        double sn, cs;
        sincos(h, &sn, &cs);
        double a = k * inv4pi * sinc;
        g = mk(-a * sn, a * cs);
      }
      double ww = Wa[i] * Wb[j];
      g = ww * g;
      gi = gi + g;
      double rb[3] = {Pb[3 * j] - cb[0], Pb[3 * j + 1] - cb[1], Pb[3 * j + 2] - cb[2]};
      for (int d = 0; d < 3; ++d) hi[d] = hi[d] + rb[d] * g;
    }
    m.M0 = m.M0 + gi;
    for (int d = 0; d < 3; ++d) {
      m.Mo[d] = m.Mo[d] + ra[d] * gi;
      m.Ms[d] = m.Ms[d] + hi[d];
    }
    m.Mos = m.Mos + (ra[0] * hi[0] + ra[1] * hi[1]) + ra[2] * hi[2];
  }
  if (touch) {
    const double* va = G.V + 3 * G.T[3 * tb];
    const double* vb = G.V + 3 * G.T[3 * tb + 1];
    const double* vc = G.V + 3 * G.T[3 * tb + 2];
    const double* nb = G.Nrm + 3 * tb;
    for (int i = 0; i < 7; ++i) {
      double r[3] = {Pa[3 * i], Pa[3 * i + 1], Pa[3 * i + 2]};
      double K0, K1[3];
      tri_potential(r, va, vb, vc, nb, K0, K1);
      double dist = nb[0] * (r[0] - va[0]) + nb[1] * (r[1] - va[1]) + nb[2] * (r[2] - va[2]);
      double K1c[3];
      for (int d = 0; d < 3; ++d) K1c[d] = K1[d] + ((r[d] - dist * nb[d]) - cb[d]) * K0;
      double w4 = Wa[i] * inv4pi;
      double ra[3] = {r[0] - ca[0], r[1] - ca[1], r[2] - ca[2]};
      m.M0.re += w4 * K0;
      for (int d = 0; d < 3; ++d) {
        m.Mo[d].re += w4 * K0 * ra[d];
        m.Ms[d].re += w4 * K1c[d];
      }
      m.Mos.re += w4 * (ra[0] * K1c[0] + ra[1] * K1c[1] + ra[2] * K1c[2]);
    }
  }
}

__device__ bool touching(const DevGeo& G, int ta, int tb) {
  const int32_t* A = G.T + 3 * ta;
  const int32_t* B = G.T + 3 * tb;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (A[i] == B[j]) return true;
  return false;
}

__device__ void pair_moments(const DevGeo& G, int ta, int tb, double k, Mom& m) {
  bool t = touching(G, ta, tb);
  raw_moments(G, ta, tb, t, k, m);
  if (t) {
    Mom s;
    raw_moments(G, tb, ta, true, k, s);
    m.M0 = 0.5 * (m.M0 + s.M0);
    for (int d = 0; d < 3; ++d) {
      cx<double> mo = 0.5 * (m.Mo[d] + s.Ms[d]);
      cx<double> ms = 0.5 * (m.Ms[d] + s.Mo[d]);
      m.Mo[d] = mo;
      m.Ms[d] = ms;
    }
    m.Mos = 0.5 * (m.Mos + s.Mos);
  }
}

// Z entry between box-order slots u (test) and v (source).
__device__ cx<double> z_entry(const DevGeo& G, const DevBasis& B, int u, int v, double k, double w2e) {
  const double mu0 = 4.0e-7 * 3.14159265358979323846;
  const bool ur = B.perm[u] < B.ne;
  const bool vr = B.perm[v] < B.ne;
  cx<double> z = mk(0.0, 0.0);
  Mom m;
  if (ur && vr) {
    for (int a = 0; a < 2; ++a) {
      int ta = B.tri[2 * u + a];
      const double* ca = G.C + 3 * ta;
      const double* p = G.V + 3 * B.fv[2 * u + a];
      double pa[3] = {p[0] - ca[0], p[1] - ca[1], p[2] - ca[2]};
      for (int b = 0; b < 2; ++b) {
        int tb = B.tri[2 * v + b];
        const double* cb = G.C + 3 * tb;
        const double* q = G.V + 3 * B.fv[2 * v + b];
        double pb[3] = {q[0] - cb[0], q[1] - cb[1], q[2] - cb[2]};
        pair_moments(G, ta, tb, k, m);
        // (r-p).(r'-q) = (r-ca - pa).(r'-cb - pb)
        cx<double> I1 = m.Mos;
        I1 = I1 - ((pa[0] * m.Ms[0] + pa[1] * m.Ms[1]) + pa[2] * m.Ms[2]);
        I1 = I1 - ((pb[0] * m.Mo[0] + pb[1] * m.Mo[1]) + pb[2] * m.Mo[2]);
        I1 = I1 + (pa[0] * pb[0] + pa[1] * pb[1] + pa[2] * pb[2]) * m.M0;
        z = z + (B.s[2 * u + a] * B.s[2 * v + b]) * I1;
      }
    }
    z = mu0 * z;
  } else if (ur && !vr) {
    int tp = B.tri[2 * v];
    for (int a = 0; a < 2; ++a) {
      pair_moments(G, B.tri[2 * u + a], tp, k, m);
      z = z + B.d[2 * u + a] * m.M0;
    }
  } else if (!ur && vr) {
    int tq = B.tri[2 * u];
    for (int b = 0; b < 2; ++b) {
      pair_moments(G, tq, B.tri[2 * v + b], k, m);
      z = z + B.d[2 * v + b] * m.M0;
    }
  } else {
    pair_moments(G, B.tri[2 * u], B.tri[2 * v], k, m);
    z = w2e * m.M0;
  }
  return z;
}

// Entry of the scalar operator S_qp = <P_q, int P_p g> between the
// triangles of the pulses at box-order slots u and v.
__device__ cx<double> s_entry(const DevGeo& G, const DevBasis& B, int u, int v, double k) {
  Mom m;
  pair_moments(G, B.tri[2 * u], B.tri[2 * v], k, m);
  return m.M0;
}

// One workgroup per stored block (a, b) of a near structure: RWG-RWG
// entries Z_mn (kind 0) or triangle-triangle entries S_qp (kind 1).
template <typename TN>
__global__ void __launch_bounds__(256) k_near_fill(DevGeo G, DevBasis B, DevNear NB, cx<TN>* out,
                                                   double k, double w2e, int32_t blk0) {
  const int blk = blk0 + blockIdx.x;
  const int a = NB.blk_a[blk], b = NB.blk_b[blk];
  const int ua = NB.ubase[a], na = NB.slot_ptr[a + 1] - NB.slot_ptr[a];
  const int ub = NB.ubase[b], nb = NB.slot_ptr[b + 1] - NB.slot_ptr[b];
  cx<TN>* o = out + NB.blk_off[blk];
  const int ldz = nb | 1;  // odd row stride of the stored blocks
  for (int e = threadIdx.x; e < na * nb; e += blockDim.x) {
    int i = e / nb, j = e - i * nb;
    cx<double> z = NB.kind == 0 ? z_entry(G, B, ua + i, ub + j, k, w2e) : s_entry(G, B, ua + i, ub + j, k);
    o[(size_t)i * ldz + j] = mk((TN)z.re, (TN)z.im);
  }
}

// Self blocks Z_bb of the finest boxes in FP64 (box order, row-major
// nb x nb at off[b]), for the solver's block-diagonal preconditioner.
__global__ void __launch_bounds__(256) k_diag_blocks(DevGeo G, DevBasis B, const int32_t* __restrict__ box_ptr,
                                                     const int64_t* __restrict__ off, cx<double>* __restrict__ out,
                                                     double k, double w2e) {
  const int b = blockIdx.x;
  const int u0 = box_ptr[b], nb = box_ptr[b + 1] - u0;
  cx<double>* o = out + off[b];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, j = e - i * nb;
    o[e] = z_entry(G, B, u0 + i, u0 + j, k, w2e);
  }
}

// Diagonal entries Z_uu (FP64) for the equilibration of the solver.
__global__ void k_diag(DevGeo G, DevBasis B, double* diag_abs, double k, double w2e) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= B.N) return;
  cx<double> z = z_entry(G, B, u, u, k, w2e);
  diag_abs[u] = sqrt(z.re * z.re + z.im * z.im);
}

// ---------------------------------------------------------------------------
// SpMM over the stored upper-triangle blocks.  For block (a, b) the row part
// r = Z_ab x_b goes to the partial slot of its rows and, for a < b, the
// transposed part c = Z_ab^T x_a (Z is symmetric) to a column slot.  Work
// unit = one row panel of one block (at most 16 KiB of entries), so large
// blocks spread over several workgroups.  The grid is persistent: each
// workgroup walks the panels blockIdx.x, blockIdx.x + gridDim.x, ... and
// holds the next panel's 16-byte loads (and its first right-hand-side
// group) in registers while it computes the current one from LDS, so the
// HBM stream never waits for the arithmetic.  Rows are stored with an odd
// stride (nb | 1), so one-row-per-lane LDS reads are bank-conflict free.
// For each group of RC of the W columns, threads 0..127 form the row sums
// (one row each) and threads 128..255 the column sums (one column each,
// into the panel's own column slot).  The reception kernel adds the slots
// in a fixed order: no atomics, bitwise reproducible, and each column's
// arithmetic is the same for any W, RC or grid size.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

// acc[r] += sum_{k0 <= k < k1} zp[k * zs] * xs[k * RC + r], in order of k,
// with UB LDS reads in flight per step.
template <typename TN, int RC, int UB>
__device__ inline void near_dot(const cx<TN>* zp, int zs, const cx<TN>* xs, int k0, int k1, cx<TN> (&acc)[RC]) {
  int k = k0;
  for (; k + UB <= k1; k += UB) {
    cx<TN> z[UB], xv[UB][RC];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      z[u] = zp[(size_t)(k + u) * zs];
#pragma unroll
      for (int r = 0; r < RC; ++r) xv[u][r] = xs[(k + u) * RC + r];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int r = 0; r < RC; ++r) cfma(acc[r], z[u], xv[u][r]);
  }
  for (; k < k1; ++k) {
    const cx<TN> z = zp[(size_t)k * zs];
#pragma unroll
    for (int r = 0; r < RC; ++r) cfma(acc[r], z, xs[k * RC + r]);
  }
}

// Descriptor of panel `task` from the dword that lane (tid mod 8) loaded.
__device__ inline NearTaskDesc near_desc(int32_t w) {
  NearTaskDesc d;
  d.off = (int64_t)(uint32_t)__builtin_amdgcn_readlane(w, 0) | ((int64_t)__builtin_amdgcn_readlane(w, 1) << 32);
  d.v0 = __builtin_amdgcn_readlane(w, 2);
  d.nb = __builtin_amdgcn_readlane(w, 3);
  d.ua = __builtin_amdgcn_readlane(w, 4);
  d.nr = __builtin_amdgcn_readlane(w, 5);
  d.prow = __builtin_amdgcn_readlane(w, 6);
  d.pcol = __builtin_amdgcn_readlane(w, 7);
  return d;
}

template <typename TN, int RC>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(RC == 1 && sizeof(TN) == 4 ? 8 : 1))) k_near_spmm(DevNear NB, const cx<TN>* __restrict__ Z,
                                                   const cx<TN>* __restrict__ xb, int ldx,
                                                   cx<TN>* __restrict__ part, int W) {
  constexpr int ZCAP = sizeof(TN) == 4 ? 2048 : 1024;  // 16 KiB panel
  constexpr int EPV = 16 / sizeof(cx<TN>);             // entries per 16-byte load
  constexpr int NV = ZCAP / EPV / 256;                 // 16-byte loads per thread
  constexpr int UB = 4;                                // LDS read batch of the inner products
  __shared__ __align__(16) cx<TN> Zs[ZCAP];
  __shared__ cx<TN> xa_s[128 * RC];
  __shared__ cx<TN> xb_s[128 * RC];
  const int tid = threadIdx.x;
  const int jc = tid - 128;
  const int ntask = NB.ntask;
  // descriptors are read one dword per lane (vector loads, counted with the
  // panel loads) and broadcast with readlane
  const int32_t* TW = (const int32_t*)NB.tdesc;
  f32x4 zr[NV];
  cx<TN> ztail = mk<TN>(0, 0), xr[RC];
  // registers <- panel entries and its first column group of x
  auto fetch = [&](const NearTaskDesc& t) {
    const int cnt = t.nr * (t.nb | 1), nv = cnt / EPV;
    const f32x4* src = (const f32x4*)(Z + t.off);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (tid + 256 * v < nv) zr[v] = __builtin_nontemporal_load(src + tid + 256 * v);
    if (EPV == 2 && (cnt & 1) && tid == 0) ztail = Z[t.off + cnt - 1];
    const int64_t xrow = tid < 128 ? (tid < t.nb ? t.v0 + tid : -1) : (t.pcol >= 0 && jc < t.nr ? t.ua + jc : -1);
#pragma unroll
    for (int r = 0; r < RC; ++r)
      xr[r] = xrow >= 0 && r < W ? xb[xrow * ldx + r] : mk<TN>(0, 0);
  };
  int task = blockIdx.x;
  if (task >= ntask) return;
  NearTaskDesc t = near_desc(TW[(size_t)task * 8 + (tid & 7)]);
  fetch(t);
  int next = task + gridDim.x;
  int32_t wn = TW[(size_t)min(next, ntask - 1) * 8 + (tid & 7)];
  for (;;) {
    // registers -> LDS for the current panel (the previous panel's readers
    // are past the barrier at the end of its last column group)
    const int ldz = t.nb | 1;  // odd row stride: the row reads below are bank-conflict free
    {
      const int cnt = t.nr * ldz, nv = cnt / EPV;
      f32x4* dst = (f32x4*)Zs;
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (tid + 256 * v < nv) dst[tid + 256 * v] = zr[v];
      if (EPV == 2 && (cnt & 1) && tid == 0) Zs[cnt - 1] = ztail;
      if (tid < 128) {
        if (tid < t.nb)
#pragma unroll
          for (int r = 0; r < RC; ++r) xb_s[tid * RC + r] = xr[r];
      } else if (t.pcol >= 0 && jc < t.nr) {
#pragma unroll
        for (int r = 0; r < RC; ++r) xa_s[jc * RC + r] = xr[r];
      }
    }
    const bool more = next < ntask;
    const NearTaskDesc tn = near_desc(wn);
    if (more) fetch(tn);  // in flight while this panel is computed
    const int next2 = next + gridDim.x;
    wn = TW[(size_t)min(next2, ntask - 1) * 8 + (tid & 7)];
    for (int c0 = 0; c0 < W; c0 += RC) {
      if (c0 > 0) {
        __syncthreads();  // the previous group's x staging is consumed
        if (tid < 128) {
          if (tid < t.nb)
#pragma unroll
            for (int r = 0; r < RC; ++r)
              xb_s[tid * RC + r] = c0 + r < W ? xb[(size_t)(t.v0 + tid) * ldx + c0 + r] : mk<TN>(0, 0);
        } else if (t.pcol >= 0 && jc < t.nr) {
#pragma unroll
          for (int r = 0; r < RC; ++r)
            xa_s[jc * RC + r] = c0 + r < W ? xb[(size_t)(t.ua + jc) * ldx + c0 + r] : mk<TN>(0, 0);
        }
      }
      __syncthreads();
      // one thread per row (threads 0..127) or column (128..255)
      const bool is_row = tid < 128;
      const int idx = is_row ? tid : jc;
      if (is_row ? idx < t.nr : (t.pcol >= 0 && idx < t.nb)) {
        cx<TN> acc[RC];
#pragma unroll
        for (int r = 0; r < RC; ++r) acc[r] = mk<TN>(0, 0);
        if (is_row)
          near_dot<TN, RC, UB>(Zs + (size_t)idx * ldz, 1, xb_s, 0, t.nb, acc);
        else
          near_dot<TN, RC, UB>(Zs + idx, ldz, xa_s, 0, t.nr, acc);
        cx<TN>* o = part + ((size_t)(is_row ? t.prow : t.pcol) + idx) * W + c0;
#pragma unroll
        for (int r = 0; r < RC; ++r)
          if (c0 + r < W) o[r] = acc[r];
      }
    }
    if (!more) break;
    __syncthreads();  // every reader of Zs / x staging is done
    t = tn;
    next = next2;
  }
}

// ---------------------------------------------------------------------------
// Batched FP32 near field on the matrix cores (passes of at least NM_COLS
// right-hand sides).  Same persistent panel stream as k_near_spmm; for each block of
// NM_COLS right-hand-side columns the row part Z x_b and the column part
// Z^T x_a are complex GEMMs in v_mfma_f32_16x16x4 tiles (four real products
// per complex one): waves 0 and 1 take the row tiles of the panel, waves 2
// and 3 its column tiles, both reading the panel and the staged x block
// from LDS.  Operand layout of v_mfma_f32_16x16x4 (64 lanes): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; result register v of
// lane l is D[4 (l / 16) + v][l % 16].
// ---------------------------------------------------------------------------
typedef float f32x4m __attribute__((ext_vector_type(4)));  // v_mfma_f32 accumulator
constexpr int NM_COLS = 16;

__global__ void __launch_bounds__(256) k_near_mspmm(DevNear NB, const cx<float>* __restrict__ Z,
                                                    const cx<float>* __restrict__ xb, int ldx,
                                                    cx<float>* __restrict__ part, int W) {
  constexpr int ZCAP = 2048;  // 16 KiB panel
  constexpr int NV = ZCAP / 2 / 256;
  __shared__ __align__(16) cx<float> Zs[ZCAP];
  __shared__ cx<float> xa_s[128 * NM_COLS];
  __shared__ cx<float> xb_s[128 * NM_COLS];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, kq = lane >> 4, jl = lane & 15;
  const int ntask = NB.ntask;
  const int32_t* TW = (const int32_t*)NB.tdesc;
  f32x4 zr[NV];
  cx<float> ztail = mk<float>(0, 0);
  auto fetch = [&](const NearTaskDesc& t) {
    const int cnt = t.nr * (t.nb | 1), nv = cnt / 2;
    const f32x4* src = (const f32x4*)(Z + t.off);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (tid + 256 * v < nv) zr[v] = __builtin_nontemporal_load(src + tid + 256 * v);
    if ((cnt & 1) && tid == 0) ztail = Z[t.off + cnt - 1];
  };
  int task = blockIdx.x;
  if (task >= ntask) return;
  NearTaskDesc t = near_desc(TW[(size_t)task * 8 + (tid & 7)]);
  fetch(t);
  int next = task + gridDim.x;
  int32_t wn = TW[(size_t)min(next, ntask - 1) * 8 + (tid & 7)];
  for (;;) {
    const int ldz = t.nb | 1;
    {
      const int cnt = t.nr * ldz, nv = cnt / 2;
      f32x4* dst = (f32x4*)Zs;
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (tid + 256 * v < nv) dst[tid + 256 * v] = zr[v];
      if ((cnt & 1) && tid == 0) Zs[cnt - 1] = ztail;
    }
    const bool more = next < ntask;
    const NearTaskDesc tn = near_desc(wn);
    if (more) fetch(tn);  // in flight while this panel is multiplied
    const int next2 = next + gridDim.x;
    wn = TW[(size_t)min(next2, ntask - 1) * 8 + (tid & 7)];
    const bool offd = t.pcol >= 0;
    for (int c0 = 0; c0 < W; c0 += NM_COLS) {
      if (c0 > 0) __syncthreads();  // the previous block's x staging is consumed
      for (int e = tid; e < 128 * NM_COLS; e += blockDim.x) {
        const int k = e / NM_COLS, j = e - k * NM_COLS;
        const bool cj = c0 + j < W;
        xb_s[e] = k < t.nb && cj ? xb[(size_t)(t.v0 + k) * ldx + c0 + j] : mk<float>(0, 0);
        xa_s[e] = offd && k < t.nr && cj ? xb[(size_t)(t.ua + k) * ldx + c0 + j] : mk<float>(0, 0);
      }
      __syncthreads();
      // rows (w < 2): tiles of panel rows against x_b; columns (w >= 2):
      // tiles of panel columns against x_a
      const bool rows = w < 2;
      const int nti = rows ? (t.nr + 15) >> 4 : (offd ? (t.nb + 15) >> 4 : 0);
      const int nk = rows ? t.nb : t.nr;
      const cx<float>* xs = rows ? xb_s : xa_s;
      for (int ti = w & 1; ti < nti; ti += 2) {
        f32x4m are = {0.f, 0.f, 0.f, 0.f}, aim = {0.f, 0.f, 0.f, 0.f};
        const int i = ti * 16 + jl;  // panel row (rows) or column (columns) of this lane's A
        const bool iok = i < (rows ? t.nr : t.nb);
        for (int k0 = 0; k0 < nk; k0 += 4) {
          const int k = k0 + kq;
          const bool ok = iok && k < nk;
          const cx<float> a = ok ? Zs[rows ? i * ldz + k : k * ldz + i] : mk<float>(0, 0);
          const cx<float> bx = k < nk ? xs[k * NM_COLS + jl] : mk<float>(0, 0);
          are = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, bx.re, are, 0, 0, 0);
          are = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.im, bx.im, are, 0, 0, 0);
          aim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, bx.im, aim, 0, 0, 0);
          aim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.im, bx.re, aim, 0, 0, 0);
        }
        const int base = rows ? t.prow : t.pcol, lim = rows ? t.nr : t.nb;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ii = ti * 16 + 4 * kq + v;
          if (ii < lim && c0 + jl < W) part[((size_t)base + ii) * W + c0 + jl] = mk(are[v], aim[v]);
        }
      }
    }
    if (!more) break;
    __syncthreads();  // every reader of Zs / x staging is done
    t = tn;
    next = next2;
  }
}

// ------------------------------------------------------------- launchers --
constexpr int kMaxDevices = 64;

// Workgroups of 256 threads of `kernel` resident at once on device dev.
static hipError_t resident_workgroups(const void* kernel, int dev, int& out) {
  int per_cu = 0, ncu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  out = std::max(1, per_cu) * std::max(1, ncu);
  return hipSuccess;
}

template <typename TN>
hipError_t launch_near_fill(const DevGeo& G, const DevBasis& B, const DevNear& NB, void* out,
                            double k, double w2e, hipStream_t st) {
  const int chunk = 4096;
  for (int b0 = 0; b0 < NB.nblk; b0 += chunk) {
    int n = NB.nblk - b0 < chunk ? NB.nblk - b0 : chunk;
    hipLaunchKernelGGL(k_near_fill<TN>, dim3(n), dim3(256), 0, st, G, B, NB, (cx<TN>*)out, k, w2e, b0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
template hipError_t launch_near_fill<float>(const DevGeo&, const DevBasis&, const DevNear&, void*,
                                            double, double, hipStream_t);
template hipError_t launch_near_fill<double>(const DevGeo&, const DevBasis&, const DevNear&, void*,
                                             double, double, hipStream_t);

hipError_t launch_diag_blocks(const DevGeo& G, const DevBasis& B, const int32_t* box_ptr, const int64_t* off,
                              int nbox, void* out, double k, double w2e, hipStream_t st) {
  if (nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_blocks, dim3(nbox), dim3(256), 0, st, G, B, box_ptr, off, (cx<double>*)out, k, w2e);
  return hipGetLastError();
}

hipError_t launch_diag(const DevGeo& G, const DevBasis& B, double* diag_abs, double k, double w2e,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_diag, dim3((B.N + 127) / 128), dim3(128), 0, st, G, B, diag_abs, k, w2e);
  return hipGetLastError();
}

// W columns per pass (x: [slots][ldx] in the structure's slot order, part:
// [partial slot][W]); rc: widest register group (1, 2 or 4); mfma: FP32
// entries on the matrix cores (the caller's choice, so that both structures
// of one pass switch together).
template <typename TN>
hipError_t launch_near_spmm(const DevNear& NB, const void* Z, const void* xb, int ldx, void* part, int W, int rc,
                            bool mfma, hipStream_t st) {
  if (NB.ntask == 0) return hipSuccess;
  if (W < 1 || (rc != 1 && rc != 2 && rc != 4)) return hipErrorInvalidValue;
  // persistent grids: as many workgroups as fit on the current device at
  // once (cached per kernel and device)
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (sizeof(TN) == 4 && mfma) {
    static int wgs[kMaxDevices] = {};
    if (wgs[dev] == 0 && (e = resident_workgroups((const void*)k_near_mspmm, dev, wgs[dev])) != hipSuccess) return e;
    hipLaunchKernelGGL(k_near_mspmm, dim3(std::min(NB.ntask, wgs[dev])), dim3(256), 0, st, NB,
                       (const cx<float>*)Z, (const cx<float>*)xb, ldx, (cx<float>*)part, W);
    return hipGetLastError();
  }
  const int g = W >= 4 && rc >= 4 ? 4 : (W >= 2 && rc >= 2 ? 2 : 1);
#define NS(G_)                                                                                      \
  do {                                                                                              \
    static int wgs[kMaxDevices] = {};                                                               \
    if (wgs[dev] == 0 &&                                                                            \
        (e = resident_workgroups((const void*)k_near_spmm<TN, G_>, dev, wgs[dev])) != hipSuccess)   \
      return e;                                                                                     \
    hipLaunchKernelGGL((k_near_spmm<TN, G_>), dim3(std::min(NB.ntask, wgs[dev])), dim3(256), 0, st, NB, \
                       (const cx<TN>*)Z, (const cx<TN>*)xb, ldx, (cx<TN>*)part, W);                 \
  } while (0)
  if (g == 1) NS(1); else if (g == 2) NS(2); else NS(4);
#undef NS
  return hipGetLastError();
}
template hipError_t launch_near_spmm<float>(const DevNear&, const void*, const void*, int, void*, int, int,
                                            bool, hipStream_t);
template hipError_t launch_near_spmm<double>(const DevNear&, const void*, const void*, int, void*, int, int,
                                             bool, hipStream_t);

}  // namespace pie
