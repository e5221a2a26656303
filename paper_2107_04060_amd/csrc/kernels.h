// Launch wrappers of the device kernels (kernels.hip, vanka.hip, bsr.hip, transfer.hip,
// krylov.hip).  All launches go to `st`.
#pragma once
#include "common.h"

namespace biot {

template <typename T>
struct DevPatchClass {
    T Ainv[8][8];
    T H[8][6];
    T G[6][6];
    T Q[6][6];
    T c[6];
    int present[PATCH];
};


// Device view of one mesh level.
template <typename T>
struct LevelView {
    Layout L;
    const T* kinv;                 // 2 planes: 1/K of L and U triangles (padded)
    const T* coef;                 // operator stencil coefficients (structure.h order, device)
    const DevPatchClass<double>* cls; // 9 Vanka classes (variable-K elimination in FP64)
    const double* wblk;            // 6 x 2 x 2 RT0-mass blocks of the star triangles (1/K = 1)
    const DevPatchClass<float>* cls32; // the same in FP32, for the FP32 elimination
    const float* wblk32;
    bool patch32;                  // variable-K Vanka eliminations in FP32 (FP32 vectors only)
    const T* uinv;                 // 9 x 8 x 8 displacement-patch inverses (BSR; identity on absent DoFs)
    const T* bsrd;                 // BSR diagonal data, 5 planes (k_bsr_wdiag / k_bsr_sdiag)
    const double* minv;            // 9 x 20 x 20 full patch inverses (uniform K), or null
    const double* fac;             // variable K: the FP64 factors of every vertex patch (PFAC planes of
                                   // the level's slot layout, patch_factor), or null
};

// vector plumbing
void launch_fill(double* x, long long n, double v, hipStream_t st);
void launch_fill(float* x, long long n, float v, hipStream_t st);
// y += x over n entries
template <typename T>
void launch_add(T* y, const T* x, long long n, hipStream_t st);
void launch_pack(const double* canon, double* padded, const Layout& L, const Canon& C, hipStream_t st);
void launch_unpack(const double* padded, double* canon, const Layout& L, const Canon& C, hipStream_t st);
void launch_convert(const double* src, float* dst, long long n, hipStream_t st);
void launch_convert(const float* src, double* dst, long long n, hipStream_t st);

// operator: y = A x (mode 0) or y = b - A x (mode 1)
template <typename T>
void launch_apply(const LevelView<T>& lv, const T* x, const T* b, T* y, int mode, hipStream_t st);

// Optional event pair recording the start and the end of one launch (the kernel's own
// timestamps, through hipExtLaunchKernel); instrumentation only.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};

// fused residual + additive Vanka step (Sec. 3.2.1):
//   x_out = x_in + omega * sum_l V_l^T D_l A_l^{-1} V_l (b - A x_in)
// x_in == nullptr means x_in = 0.  x_out must not alias x_in.  uniform: one patch inverse per
// vertex class (lv.minv, full inverses), 1/K = kinv_s; else per-patch elimination with lv.kinv.
// xc != nullptr: the iterate is x_in + P x_c (coarse level layout *Lc, prolongation weights
// pw), i.e. the prolongation of the coarse-grid correction is fused into the step.
// color >= 0: one colour step of the multiplicative form (only the patches of vertices of that
// colour, unweighted): codes 0..3 the four colours (i mod 2) + 2 (j mod 2), codes 4..6 the three
// colours 4 + (i + 2 j) mod 3; -1: the additive step.
template <typename T>
void launch_vanka_step(const LevelView<T>& lv, const T* x_in, const T* b, T* x_out, bool uniform, T kinv_s,
                       T omega, hipStream_t st, const T* xc = nullptr, const Layout* Lc = nullptr,
                       const T* pw = nullptr, const LaunchTiming* tm = nullptr, int color = -1);

// the permeability-dependent factors of every vertex patch of a level (variable K, FP64):
// fac[q * L.plane + slot(i, j)], q < PFAC (patch_solve.h)
void launch_patch_factors(const LevelView<double>& lv, double* fac, hipStream_t st);

// grid transfers
// (w: the NPWEIGHTS prolongation weights of structure.h, device)
template <typename T>
void launch_restrict(const Layout& Lf, const Layout& Lc, const T* rf, T* rc, const T* w, hipStream_t st);
template <typename T>
void launch_prolong_add(const Layout& Lf, const Layout& Lc, const T* xc, T* xf, const T* w, hipStream_t st);
// r_c = P^T (b - A_f x) in one launch (the fine residual is not stored); uniform: 1/K = kinv_s
template <typename T>
void launch_residual_restrict(const LevelView<T>& lf, const Layout& Lc, const T* x, const T* b, T* rc,
                              bool uniform, T kinv_s, const T* w, hipStream_t st, const LaunchTiming* tm = nullptr);

// inexact Braess-Sarazin: diagonal data of a level (1 / (tau D_w), 1 / diag(S)); cS =
// (1/M + alpha^2 / (lambda + mu)) |T|
template <typename T>
void launch_bsr_diag(const LevelView<T>& lv, T cS, T* d, hipStream_t st);
// one BSR step x <- x + omega M_BSR^{-1} (b - A x) in two launches (r, t: scratch vectors of the
// level; x_is_zero: x = 0 on entry).  xc != nullptr: the iterate is x + P x_c (coarse layout
// *Lc, prolongation weights pw), formed into xtmp (!= x) on the way; the result is in x.
// sw (optional): the pressure correction from sweeps > 1 weighted-Jacobi sweeps (weight omega_S)
// on the approximate Schur complement instead of the single step with omega_J; cS = (1/M +
// alpha^2 / (lambda + mu)) |T|; buf: 6 zero-initialized planes of the level.
// cg > 0 (instead of sweeps): the pressure correction from cg steps of diag(S_hat)-preconditioned
// conjugate gradients on S_hat from zero; buf: 10 planes, red: 2 cg_partials(L) + 3 doubles.
template <typename T>
struct SchurSweeps {
    int sweeps;
    T omega_S;
    T cS;
    T* buf;
    int cg = 0;
    double* red = nullptr;
};
// partial sums per dot product of the Schur CG on a level
int cg_partials(const Layout& L);
template <typename T>
void launch_bsr_step(const LevelView<T>& lv, T* x, const T* b, T* r, T* t, bool x_is_zero, bool uniform, T kinv_s,
                     T omega, T omega_J, const T* xc, const Layout* Lc, const T* pw, T* xtmp, hipStream_t st,
                     const SchurSweeps<T>* sw = nullptr);

// coarsest level (Ainv: the inverse of the coarsest operator, row-major)
template <typename T>
void launch_coarse_solve(const double* Ainv, int N, const int* idx, const T* b, T* x, hipStream_t st);
void launch_coarse_matrix(const Layout& L, const StencilEntry* st_tab, const int* st_off, const double* kinv,
                          const int* free_idx, const int* free_map, int N, double* A, hipStream_t st);
// dense inverse by Gauss-Jordan with partial pivoting (A destroyed; fcol: N doubles of scratch;
// *status = 1 on a zero pivot column)
void launch_gauss_jordan(double* A, double* Inv, int N, double* fcol, int* status, hipStream_t st);

// permeability
void launch_kinv_from_K(const double* K_tri, double K_scalar, double* kinv, const Layout& L, hipStream_t st);
void launch_kinv_coarsen(const double* kf, const Layout& Lf, double* kc, const Layout& Lc, hipStream_t st);
// 1/K = exp(-theta) on the finest level from per-triangle theta = ln K
void launch_kinv_from_logK(const double* theta_tri, double* kinv, const Layout& L, hipStream_t st);
// *bad (device int) = 1 if any of the n values is unusable: mode 0 a permeability (K > 0, 1/K
// finite and non-zero), mode 1 a log-permeability (|theta| < 700); else 0
void launch_check_field(const double* v, long long n, int mode, int* bad, hipStream_t st);

// Krylov BLAS-1 (FP64)
void launch_scale(double* dst, const double* src, long long n, double s, hipStream_t st);
void launch_lincomb_add(double* x, const double* Z, long long ldz, int nv, const double* y, long long n,
                        hipStream_t st);
// one classical Gram-Schmidt pass, each call two launches (partial sums, then a fixed-order
// reduction; partial: max(RED_BLOCKS x (nv + 1), 4 RED_BLOCKS) doubles).  dots: out[q] = V_q . w,
// out[nv] = w . w.  update: w -= V h, norm2 = w . w, flag (optional) = (norm2 < eta2 prev).
// host: optional mirror of the outputs (mapped memory; flag goes to host[1]).  run_if: every
// launch returns at once when *run_if == 0.
void launch_gs_dots(const double* V, long long ldv, int nv, const double* w, long long n, double* partial,
                    double* out, double* host, const double* run_if, hipStream_t st);
void launch_gs_update(double* w, const double* V, long long ldv, int nv, const double* h, long long n,
                      double* partial, double* norm2, const double* prev, double* flag, double* host,
                      const double* run_if, hipStream_t st, double eta2 = 0.5);
// the first pass's update fused with the second pass's dot products (nv <= GS_FUSED): w -= V h,
// out[q] = V_q . w (q < nv) and out[nv] = w . w of the new w; flag = (out[nv] < eta2 prev),
// mirrored to host_flag; host: optional mirror of out.  Two launches.
constexpr int GS_FUSED = 32;
void launch_gs_update_dots(double* w, const double* V, long long ldv, int nv, const double* h, long long n,
                           double* partial, double* out, double* host, const double* prev, double* flag,
                           double* host_flag, hipStream_t st, double eta2 = 0.5);
// dst = src / sqrt(*na), or / sqrt(*nb) when sel != nullptr and *sel != 0
void launch_normalize(double* dst, const double* src, long long n, const double* na, const double* nb,
                      const double* sel, hipStream_t st);

// adjoint: per-triangle  1/K_T * lam_w|_T^T  Mloc_T  w|_T  (Mloc: 2 types x 3 x 3)
void launch_grad_logK(const Layout& L, const double* x, const double* lam, const double* kinv,
                      const double* mloc, double* g_tri, hipStream_t st);

// layout export
void launch_patch_table(const Layout& L, const Canon& C, int* table, hipStream_t st);

constexpr int RED_BLOCKS = 1024;  // Gram-Schmidt partial sums: RED_BLOCKS x (vectors + 1), >= 4 RED_BLOCKS

}  // namespace biot
