// Right-hand sides, far field and the FP64 vector kernels of the GMRES solver.
#include "device.h"
#include "kernels.h"

namespace pie {

// ---------------------------------------------------------------------------
// Plane-wave right-hand side (Eqs. (1)-(2)):  b^J_m = -<f_m, A^inc>,
// b^A_q = -i w eps0 <P_q, Phi^inc>.  One thread per (unknown, RHS).
// ---------------------------------------------------------------------------
__global__ void k_rhs(DevGeo G, const double* __restrict__ s, const int32_t* __restrict__ tri,
                      const int32_t* __restrict__ fv, int ne, int nt, const double* __restrict__ khat,
                      const double* __restrict__ pol, const double* __restrict__ amp, int R, int gauge,
                      double k, double omega, cx<double>* __restrict__ b) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = ne + nt;
  if (e >= (int64_t)N * R) return;
  const int u = (int)(e / R), r = (int)(e - (int64_t)u * R);
  const double eps0 = 1.0 / (4.0e-7 * 3.14159265358979323846 * 299792458.0 * 299792458.0);
  const double c0 = 299792458.0;
  const double* kh = khat + 3 * r;
  const double* pl = pol + 3 * r;
  const cx<double> a = mk(amp[2 * r], amp[2 * r + 1]);
  cx<double> acc = mk(0.0, 0.0);
  if (u < ne) {
    for (int h = 0; h < 2; ++h) {
      const int t = tri[2 * u + h];
      const double* pv = G.V + 3 * fv[2 * u + h];
      const double sc = s[2 * u + h];
      for (int i = 0; i < 7; ++i) {
        const double* P = G.P + 21 * t + 3 * i;
        double sn, cs;
        sincos(k * (kh[0] * P[0] + kh[1] * P[1] + kh[2] * P[2]), &sn, &cs);
        cx<double> ph = mk(cs, sn) * a;
        double f[3] = {sc * (P[0] - pv[0]), sc * (P[1] - pv[1]), sc * (P[2] - pv[2])};
        cx<double> fa;
        if (gauge == 0) {
          double pr = pl[0] * P[0] + pl[1] * P[1] + pl[2] * P[2];
          double fk = f[0] * kh[0] + f[1] * kh[1] + f[2] * kh[2];
          fa = (-pr * fk / c0) * ph;
        } else {
          double fp = f[0] * pl[0] + f[1] * pl[1] + f[2] * pl[2];
          // E / (i w) = -i E / w
          fa = (fp / omega) * mk(ph.im, -ph.re);
        }
        acc = acc + G.W[7 * t + i] * fa;
      }
    }
    acc = mk(-acc.re, -acc.im);
  } else {
    const int t = u - ne;
    if (gauge == 0) {
      for (int i = 0; i < 7; ++i) {
        const double* P = G.P + 21 * t + 3 * i;
        double sn, cs;
        sincos(k * (kh[0] * P[0] + kh[1] * P[1] + kh[2] * P[2]), &sn, &cs);
        cx<double> ph = mk(cs, sn) * a;
        double pr = pl[0] * P[0] + pl[1] * P[1] + pl[2] * P[2];
        acc = acc + (G.W[7 * t + i] * -pr) * ph;
      }
      // -i w eps0 * acc
      double f = omega * eps0;
      acc = mk(f * acc.im, -f * acc.re);
    }
  }
  b[e] = acc;
}

hipError_t launch_rhs(const DevGeo& G, const double* s, const int32_t* tri, const int32_t* fv, int ne, int nt,
                      const double* khat, const double* pol, const double* amp, int R, int gauge, double k,
                      double omega, void* b, hipStream_t st) {
  int64_t n = (int64_t)(ne + nt) * R;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, G, s, tri, fv, ne, nt, khat, pol,
                     amp, R, gauge, k, omega, (cx<double>*)b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Far field F(rhat) = (i w mu0/4pi)(I - rhat rhat) . sum_n a_n int f_n
// exp(-i k rhat.r').  One workgroup per (RHS, direction); fixed-order
// block reduction.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_farfield(DevGeo G, const double* __restrict__ s,
                                                  const int32_t* __restrict__ tri, const int32_t* __restrict__ fv,
                                                  int ne, const cx<double>* __restrict__ x, int R,
                                                  const double* __restrict__ dirs, int nd, double k, double omega,
                                                  cx<double>* __restrict__ F) {
  __shared__ cx<double> red[256][3];
  const int r = blockIdx.x / nd, dd = blockIdx.x - r * nd;
  const double* rh = dirs + 3 * dd;
  cx<double> acc[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  for (int n = threadIdx.x; n < ne; n += blockDim.x) {
    const cx<double> a = x[(size_t)n * R + r];
    for (int h = 0; h < 2; ++h) {
      const int t = tri[2 * n + h];
      const double* pv = G.V + 3 * fv[2 * n + h];
      const double sc = s[2 * n + h];
      for (int i = 0; i < 7; ++i) {
        const double* P = G.P + 21 * t + 3 * i;
        double sn, cs;
        sincos(-k * (rh[0] * P[0] + rh[1] * P[1] + rh[2] * P[2]), &sn, &cs);
        cx<double> ph = (G.W[7 * t + i] * sc) * (mk(cs, sn) * a);
        for (int c = 0; c < 3; ++c) acc[c] = acc[c] + (P[c] - pv[c]) * ph;
      }
    }
  }
  for (int c = 0; c < 3; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int c = 0; c < 3; ++c) red[threadIdx.x][c] = red[threadIdx.x][c] + red[threadIdx.x + o][c];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cx<double> J[3] = {red[0][0], red[0][1], red[0][2]};
    cx<double> rr = (rh[0] * J[0] + rh[1] * J[1]) + rh[2] * J[2];
    const double f = omega * 4.0e-7 * 3.14159265358979323846 / (4.0 * 3.14159265358979323846);
    for (int c = 0; c < 3; ++c) {
      cx<double> t = J[c] - rh[c] * rr;
      F[((size_t)r * nd + dd) * 3 + c] = mk(-f * t.im, f * t.re);  // i f t
    }
  }
}

hipError_t launch_farfield(const DevGeo& G, const double* s, const int32_t* tri, const int32_t* fv, int ne,
                           const void* x, int R, const double* dirs, int nd, double k, double omega, void* F,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_farfield, dim3(R * nd), dim3(256), 0, st, G, s, tri, fv, ne, (const cx<double>*)x, R, dirs,
                     nd, k, omega, (cx<double>*)F);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint of the far-field map: for F = Phi x as above,
//   gx[n][r] = sum_d conj(Phi[d][:, n]) . gF[r][d][:]
//            = sum_d conj(i w mu0/4pi) conj(Jn(d)) . ((I - rhat rhat) gF[r][d]),
//   Jn(d) = int f_n exp(-i k rhat_d.r') dr'.
// One thread per (RWG function, RHS); pulse rows of gx are zero.
// ---------------------------------------------------------------------------
__global__ void k_farfield_adj(DevGeo G, const double* __restrict__ s, const int32_t* __restrict__ tri,
                               const int32_t* __restrict__ fv, int ne, int nt, const cx<double>* __restrict__ gF,
                               int R, const double* __restrict__ dirs, int nd, double k, double omega,
                               cx<double>* __restrict__ gx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)(ne + nt) * R) return;
  const int n = (int)(e / R), r = (int)(e - (int64_t)n * R);
  if (n >= ne) {
    gx[e] = mk(0.0, 0.0);
    return;
  }
  const double f = omega * 4.0e-7 * 3.14159265358979323846 / (4.0 * 3.14159265358979323846);
  cx<double> acc = mk(0.0, 0.0);
  for (int dd = 0; dd < nd; ++dd) {
    const double* rh = dirs + 3 * dd;
    const cx<double>* g = gF + ((size_t)r * nd + dd) * 3;
    cx<double> gr = (rh[0] * g[0] + rh[1] * g[1]) + rh[2] * g[2];
    cx<double> gt[3];
    for (int c = 0; c < 3; ++c) gt[c] = g[c] - rh[c] * gr;
    // conj(Jn) . gt, Jn = sum W s (P - p) exp(-i k rhat.P)  -> conj(exp) = exp(+i k rhat.P)
    cx<double> sum = mk(0.0, 0.0);
    for (int h = 0; h < 2; ++h) {
      const int t = tri[2 * n + h];
      const double* pv = G.V + 3 * fv[2 * n + h];
      const double sc = s[2 * n + h];
      for (int i = 0; i < 7; ++i) {
        const double* P = G.P + 21 * t + 3 * i;
        double sn, cs;
        sincos(k * (rh[0] * P[0] + rh[1] * P[1] + rh[2] * P[2]), &sn, &cs);
        cx<double> dot = ((P[0] - pv[0]) * gt[0] + (P[1] - pv[1]) * gt[1]) + (P[2] - pv[2]) * gt[2];
        sum = sum + (G.W[7 * t + i] * sc) * (mk(cs, sn) * dot);
      }
    }
    acc = acc + sum;
  }
  // times conj(i f) = -i f
  gx[e] = mk(f * acc.im, -f * acc.re);
}

hipError_t launch_farfield_adj(const DevGeo& G, const double* s, const int32_t* tri, const int32_t* fv, int ne,
                               int nt, const void* gF, int R, const double* dirs, int nd, double k, double omega,
                               void* gx, hipStream_t st) {
  int64_t n = (int64_t)(ne + nt) * R;
  hipLaunchKernelGGL(k_farfield_adj, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, G, s, tri, fv, ne, nt,
                     (const cx<double>*)gF, R, dirs, nd, k, omega, (cx<double>*)gx);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Solver vector kernels on [N][R] complex128 blocks.
// ---------------------------------------------------------------------------
__global__ void k_scale_rows(const cx<double>* __restrict__ x, const double* __restrict__ d, int N, int R,
                             cx<double>* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * R) return;
  y[e] = d[e / R] * x[e];
}
hipError_t launch_scale_rows(const void* x, const double* d, int N, int R, void* y, hipStream_t st) {
  int64_t n = (int64_t)N * R;
  hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const cx<double>*)x, d,
                     N, R, (cx<double>*)y);
  return hipGetLastError();
}

// out[i][r] = sum_n conj(V_i[n][r]) w[n][r]; one workgroup per (i, r).
__global__ void __launch_bounds__(256) k_dots(const cx<double>* __restrict__ V, int64_t vstride,
                                              const cx<double>* __restrict__ w, int N, int R,
                                              cx<double>* __restrict__ out) {
  __shared__ cx<double> red[256];
  const int i = blockIdx.x / R, r = blockIdx.x - (blockIdx.x / R) * R;
  const cx<double>* v = V + (size_t)i * vstride;
  cx<double> acc = mk(0.0, 0.0);
  for (int n = threadIdx.x; n < N; n += blockDim.x) cfma_conj(acc, v[(size_t)n * R + r], w[(size_t)n * R + r]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)i * R + r] = red[0];
}
hipError_t launch_dots(const void* V, int64_t vstride, int nv, const void* w, int N, int R, void* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_dots, dim3(nv * R), dim3(256), 0, st, (const cx<double>*)V, vstride, (const cx<double>*)w,
                     N, R, (cx<double>*)out);
  return hipGetLastError();
}

// w[n][r] -= sum_i V_i[n][r] h[i][r]
__global__ void k_update(cx<double>* __restrict__ w, const cx<double>* __restrict__ V, int64_t vstride, int nv,
                         const cx<double>* __restrict__ h, int N, int R) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * R) return;
  const int r = (int)(e % R);
  cx<double> acc = w[e];
  for (int i = 0; i < nv; ++i) {
    cx<double> t = V[(size_t)i * vstride + e] * h[(size_t)i * R + r];
    acc = acc - t;
  }
  w[e] = acc;
}
hipError_t launch_update(void* w, const void* V, int64_t vstride, int nv, const void* h, int N, int R,
                         hipStream_t st) {
  int64_t n = (int64_t)N * R;
  hipLaunchKernelGGL(k_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (cx<double>*)w,
                     (const cx<double>*)V, vstride, nv, (const cx<double>*)h, N, R);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_norms(const cx<double>* __restrict__ w, int N, int R,
                                               double* __restrict__ out) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  double acc = 0.0;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    cx<double> v = w[(size_t)n * R + r];
    acc = fma(v.re, v.re, acc);
    acc = fma(v.im, v.im, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = sqrt(red[0]);
}
hipError_t launch_norms(const void* w, int N, int R, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norms, dim3(R), dim3(256), 0, st, (const cx<double>*)w, N, R, out);
  return hipGetLastError();
}

__global__ void k_colscale(cx<double>* __restrict__ w, const double* __restrict__ s, int N, int R) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * R) return;
  w[e] = s[e % R] * w[e];
}
hipError_t launch_colscale(void* w, const double* s, int N, int R, hipStream_t st) {
  int64_t n = (int64_t)N * R;
  hipLaunchKernelGGL(k_colscale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (cx<double>*)w, s, N, R);
  return hipGetLastError();
}

// x[n][r] += a[r] y[n][r]
__global__ void k_axpy_cols(cx<double>* __restrict__ x, const cx<double>* __restrict__ y,
                            const cx<double>* __restrict__ a, int N, int R) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * R) return;
  cfma(x[e], a[e % R], y[e]);
}
hipError_t launch_axpy_cols(void* x, const void* y, const void* a, int N, int R, hipStream_t st) {
  int64_t n = (int64_t)N * R;
  hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (cx<double>*)x,
                     (const cx<double>*)y, (const cx<double>*)a, N, R);
  return hipGetLastError();
}

__global__ void k_sub(const cx<double>* __restrict__ a, const cx<double>* __restrict__ b, int64_t n,
                      cx<double>* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  out[e] = a[e] - b[e];
}
hipError_t launch_sub(const void* a, const void* b, int N, int R, void* out, hipStream_t st) {
  int64_t n = (int64_t)N * R;
  hipLaunchKernelGGL(k_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const cx<double>*)a,
                     (const cx<double>*)b, n, (cx<double>*)out);
  return hipGetLastError();
}

// Right-hand side of the charge equation from a plane-wave one: RWG rows
// cleared, pulse rows times c.
__global__ void k_pulse_rhs(cx<double>* __restrict__ b, int64_t nj, int64_t n, cx<double> c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  b[e] = e < nj ? mk(0.0, 0.0) : c * b[e];
}
hipError_t launch_pulse_rhs(void* b, int E, int N, int R, double cre, double cim, hipStream_t st) {
  const int64_t n = (int64_t)N * R;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pulse_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (cx<double>*)b,
                     (int64_t)E * R, n, mk(cre, cim));
  return hipGetLastError();
}

// rho = i w eps0 (n.A) - eps0 sigma, per triangle and column.
__global__ void k_charge_rho(const cx<double>* __restrict__ na, const cx<double>* __restrict__ sigma, int64_t n,
                             double weps0, double eps0, cx<double>* __restrict__ rho) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const cx<double> a = na[e], s = sigma[e];
  rho[e] = mk(-weps0 * a.im - eps0 * s.re, weps0 * a.re - eps0 * s.im);
}
hipError_t launch_charge_rho(const cx<double>* na, const cx<double>* sigma, int64_t n, double weps0, double eps0,
                             void* rho, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_charge_rho, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, na, sigma, n, weps0, eps0,
                     (cx<double>*)rho);
  return hipGetLastError();
}

// Block-diagonal preconditioner: for every finest box b,
//   y[perm[u]] = sum_{v in b} Minv_b[u][v] x[perm[v]] / d[perm[v]]
// (R columns; Minv_b row-major nb x nb at off[b], box order; d NULL: 1).
__global__ void __launch_bounds__(128) k_block_prec(const cx<double>* __restrict__ x, const double* __restrict__ d,
                                                    const cx<double>* __restrict__ minv,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ box_ptr,
                                                    const int32_t* __restrict__ perm, int R,
                                                    cx<double>* __restrict__ y) {
  const int b = blockIdx.x;
  const int u0 = box_ptr[b], nb = box_ptr[b + 1] - u0;
  const cx<double>* M = minv + off[b];
  for (int e = threadIdx.x; e < nb * R; e += blockDim.x) {
    const int i = e / R, r = e - i * R;
    cx<double> acc = mk(0.0, 0.0);
    for (int j = 0; j < nb; ++j) {
      const int cv = perm[u0 + j];
      cfma(acc, M[(size_t)i * nb + j], (d ? 1.0 / d[cv] : 1.0) * x[(size_t)cv * R + r]);
    }
    y[(size_t)perm[u0 + i] * R + r] = acc;
  }
}
hipError_t launch_block_prec(const void* x, const double* d, const void* minv, const int64_t* off,
                             const int32_t* box_ptr, const int32_t* perm, int nbox, int R, void* y, hipStream_t st) {
  if (nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_prec, dim3(nbox), dim3(128), 0, st, (const cx<double>*)x, d, (const cx<double>*)minv,
                     off, box_ptr, perm, R, (cx<double>*)y);
  return hipGetLastError();
}

// x += t / d (per row), n = N R entries.
__global__ void k_add_scaled(cx<double>* __restrict__ x, const cx<double>* __restrict__ t,
                             const double* __restrict__ d, int64_t n, int R) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  x[e] = x[e] + (1.0 / d[e / R]) * t[e];
}
hipError_t launch_add_scaled(void* x, const void* t, const double* d, int N, int R, hipStream_t st) {
  const int64_t n = (int64_t)N * R;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_scaled, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (cx<double>*)x,
                     (const cx<double>*)t, d, n, R);
  return hipGetLastError();
}

}  // namespace pie
