// Host-side launchers of the HIP kernels (each launcher returns the launch
// error; kernels run asynchronously on the given stream).
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"

namespace pie {

// near.hip
template <typename TN>
hipError_t launch_near_fill(const DevGeo& G, const DevBasis& B, const DevNear& NB, void* out, double k,
                            double w2e, hipStream_t st);
hipError_t launch_diag(const DevGeo& G, const DevBasis& B, double* diag_abs, double k, double w2e,
                       hipStream_t st);
// FP64 self blocks of the finest boxes (row-major nb x nb at off[b], box order).
hipError_t launch_diag_blocks(const DevGeo& G, const DevBasis& B, const int32_t* box_ptr, const int64_t* off,
                              int nbox, void* out, double k, double w2e, hipStream_t st);
// W columns per pass, register groups of at most rc columns; mfma: FP32
// entries on the matrix cores.
template <typename TN>
hipError_t launch_near_spmm(const DevNear& NB, const void* Z, const void* xb, int ldx, void* part, int W, int rc,
                            bool mfma, hipStream_t st);

// far.hip
size_t aggregate_smem(int maxinc, int Q, int nsplit, int RC, int tf_bytes);
size_t receive_smem(int maxinc, int Q, int maxjoin, int RC, int tf_bytes);
// Per-incidence moment table M[ninc][Qh][4] (M0, M1x, M1y, M1z) at the finest
// level, for the first Qh samples (the others are antipodes: M(q) = conj
// M(anti[q])).
template <typename TF>
hipError_t launch_moments(const double* pw, int ninc, const double* khat64, int Qh, double kappa, void* M,
                          hipStream_t st);
// W right-hand-side columns per pass, register groups of at most rc columns.
template <typename TF>
hipError_t launch_aggregate(const DevInc& I, int nb, int maxinc, const void* x, int ldx, int W, int rc,
                            const void* M, const int32_t* anti, int Q, int Qh, double w2e, int conjx, int nsplit,
                            void* S, hipStream_t st);
// Filter tables (Ft for the upward, F for the downward shift) carry SQT
// trailing zeros.
// force_mfma: FP64 shifts on the matrix cores whatever the level's size.
template <typename TF>
hipError_t launch_shift_up(const DevLevel& Lp, const DevLevel& Lc, const void* Sc, void* Sp, const void* Ft,
                           const void* ph, int Q, int R, bool force_mfma, hipStream_t st);
template <typename TF>
hipError_t launch_shift_down(const DevLevel& Lc, const void* Gp, void* Gc, const void* F, const void* ph, int Q,
                             int R, bool force_mfma, hipStream_t st);
// T: translation values [TRANSLATE_OFFSETS][Q].
template <typename TF>
hipError_t launch_translate(const DevLevel& Lv, const void* S, const void* T, void* Gout, int Q, int R,
                            hipStream_t st);
// Translations of n levels (arrays of n) in one launch where possible.
template <typename TF>
hipError_t launch_translate_levels(const DevLevel* lv, const void* const* S, const void* const* T, void* const* G,
                                   int n, int Q, int R, hipStream_t st);
// Reception + near join: RWG rows and pulse rows of y (canonical, FP64,
// leading dimension ldy) and the per-triangle potentials phi [T][W].
template <typename TF, typename TN>
hipError_t launch_receive(const DevInc& I, const DevBasis& B, const DevNear& NJ, const DevNear& NT, int nb,
                          int maxinc, int maxjoin, const void* Gin, const void* M, const int32_t* anti, int Q, int Qh,
                          const void* partJ, const void* partT, int W, int rc, int flags, void* y, int ldy,
                          void* phi, hipStream_t st);
// Near-field inputs: RWG slots xJ [E][W] and triangle slots xT [T][2W] (x_A, u).
template <typename TN>
hipError_t launch_near_in(const void* x, int ldx, const int32_t* permJ, const int32_t* permT, const DevTriDiv& td,
                          double w2e, int W, int conjx, void* xJ, void* xT, hipStream_t st);
// y[m] += sum_h 2 cs[m][h] phi[tri[m][h]] for the ne RWG rows.
hipError_t launch_div_test(const int32_t* tri, const double* cs, const void* phi, int ne, int W, void* y, int ldy,
                           hipStream_t st);

// aux.hip
hipError_t launch_rhs(const DevGeo& G, const double* basis_canon_s, const int32_t* tri_canon,
                      const int32_t* fv_canon, int ne, int nt, const double* khat, const double* pol,
                      const double* amp, int R, int gauge, double k, double omega, void* b, hipStream_t st);
hipError_t launch_farfield(const DevGeo& G, const double* s_canon, const int32_t* tri_canon,
                           const int32_t* fv_canon, int ne, const void* x, int R, const double* dirs, int nd,
                           double k, double omega, void* F, hipStream_t st);
hipError_t launch_farfield_adj(const DevGeo& G, const double* s_canon, const int32_t* tri_canon,
                               const int32_t* fv_canon, int ne, int nt, const void* gF, int R, const double* dirs,
                               int nd, double k, double omega, void* gx, hipStream_t st);
// y[:, r] = alpha_r-free helpers for the solver (complex128, [N][R]).
hipError_t launch_scale_rows(const void* x, const double* d, int N, int R, void* y, hipStream_t st);
hipError_t launch_dots(const void* V, int64_t vstride, int nv, const void* w, int N, int R, void* out,
                       hipStream_t st);
hipError_t launch_update(void* w, const void* V, int64_t vstride, int nv, const void* h, int N, int R,
                         hipStream_t st);
hipError_t launch_norms(const void* w, int N, int R, double* out, hipStream_t st);
hipError_t launch_colscale(void* w, const double* s, int N, int R, hipStream_t st);
hipError_t launch_axpy_cols(void* x, const void* y, const void* a, int N, int R, hipStream_t st);
hipError_t launch_sub(const void* a, const void* b, int N, int R, void* out, hipStream_t st);
// Charge equation (pulse-pulse block): b <- RWG rows cleared, pulse rows
// times (cre + i cim); rho = i weps0 na - eps0 sigma, n entries.
// Block-diagonal preconditioner y = Minv (x / d) through the box permutation,
// and x += t / d.
hipError_t launch_block_prec(const void* x, const double* d, const void* minv, const int64_t* off,
                             const int32_t* box_ptr, const int32_t* perm, int nbox, int R, void* y, hipStream_t st);
hipError_t launch_add_scaled(void* x, const void* t, const double* d, int N, int R, hipStream_t st);
hipError_t launch_pulse_rhs(void* b, int E, int N, int R, double cre, double cim, hipStream_t st);
hipError_t launch_charge_rho(const cx<double>* na, const cx<double>* sigma, int64_t n, double weps0, double eps0,
                             void* rho, hipStream_t st);

}  // namespace pie
