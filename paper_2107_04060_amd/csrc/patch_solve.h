// Vanka patch solve (Sec. 3.2.1), shared by the device kernels and the host set-up.
//
// Patch system of a vertex patch, by block elimination onto the six pressures:
//   [[A, 0, Bh^T], [0, W, Q^T], [Bh, Q, -C]] (xu, xw, xp) = (ru, rw, rp)
//   S xp = Bh A^-1 ru + Q W^-1 rw - rp,  S = C + Bh A^-1 Bh^T + Q W^-1 Q^T  (SPD),
//   xu = A^-1 (ru - Bh^T xp),  xw = W^-1 (rw - Q^T xp).
// The pressure constant on the star is an exact eigenvector of S with eigenvalue (1/M)|T|
// (the patch velocities carry no net flux of it): its coefficient is solved for in closed
// form, gamma = -sum(rp) / sum(c), and S is made well conditioned by a rank-one shift on
// that direction before the Cholesky factorization.  The factorizations depend on the
// permeability only (patch_factor); a relaxation step applies them (patch_apply).
#pragma once
#include "kernels.h"

#include <cmath>
#include <type_traits>

namespace biot {

// Keeps the class-data and residual reads of one phase of an FP64 patch solve from being hoisted
// into an earlier phase, where they would all be live at once (an empty asm statement with a
// memory clobber: no instruction).  The FP32 solve fits its registers without it.
#define BIOT_PHASE_FENCE()                                        \
    do {                                                          \
        if constexpr (sizeof(T) == 8) __asm__ volatile("" ::: "memory"); \
    } while (0)

// packed lower triangle of a symmetric 6 x 6 matrix
__host__ __device__ constexpr int tri6(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// Cholesky factor L (A = L L^T) in place, with 1 / L[j][j] stored on the diagonal so that the
// triangular solves multiply instead of divide
template <typename T>
__host__ __device__ inline void chol6p(T a[21]) {
#pragma unroll
    for (int jj = 0; jj < 6; ++jj) {
        T d = a[tri6(jj, jj)];
#pragma unroll
        for (int k = 0; k < jj; ++k) d -= a[tri6(jj, k)] * a[tri6(jj, k)];
        const T inv = (T)1 / sqrt(d);
        a[tri6(jj, jj)] = inv;
#pragma unroll
        for (int ii = jj + 1; ii < 6; ++ii) {
            T s = a[tri6(ii, jj)];
#pragma unroll
            for (int k = 0; k < jj; ++k) s -= a[tri6(ii, k)] * a[tri6(jj, k)];
            a[tri6(ii, jj)] = s * inv;
        }
    }
}

// v <- L^-1 v
template <typename T>
__host__ __device__ inline void fwd6p(const T l[21], T v[6]) {
#pragma unroll
    for (int ii = 0; ii < 6; ++ii) {
        T s = v[ii];
#pragma unroll
        for (int k = 0; k < ii; ++k) s -= l[tri6(ii, k)] * v[k];
        v[ii] = s * l[tri6(ii, ii)];
    }
}

// v <- L^-T v
template <typename T>
__host__ __device__ inline void bwd6p(const T l[21], T v[6]) {
#pragma unroll
    for (int ii = 5; ii >= 0; --ii) {
        T s = v[ii];
#pragma unroll
        for (int k = ii + 1; k < 6; ++k) s -= l[tri6(k, ii)] * v[k];
        v[ii] = s * l[tri6(ii, ii)];
    }
}

// 1/K of star triangle k from an array or from an accessor kv(k) (read where it is used)
template <typename T, typename KV>
__host__ __device__ inline T kv_at(const KV& kv, int k) {
    if constexpr (std::is_invocable_v<const KV&, int>)
        return kv(k);
    else
        return kv[k];
}

// Sparsity of W and of its Cholesky factor in slot order.  W couples two star edges only through
// the star triangle holding both (star_wpair): the six edges form a cycle.  Eliminating in slot
// order fills three more pairs; the other six entries of the packed factor stay zero, and the
// factorization and substitutions below skip them (the same values as the dense forms, whose
// skipped terms are exact zeros).
struct WPattern {
    bool nz[6][6];
};
__host__ __device__ constexpr WPattern w_pattern() {
    WPattern P{};
    for (int i = 0; i < 6; ++i) P.nz[i][i] = true;
    for (int k = 0; k < 6; ++k) {
        const int a = star_wpair(k, 0), b = star_wpair(k, 1);
        P.nz[a][b] = P.nz[b][a] = true;
    }
    for (int j = 0; j < 6; ++j)                     // symbolic elimination, column j
        for (int i = j + 1; i < 6; ++i)
            for (int l = j + 1; l < 6; ++l)
                if (P.nz[i][j] && P.nz[l][j]) P.nz[i][l] = P.nz[l][i] = true;
    return P;
}
__host__ __device__ constexpr bool wnz(int i, int j) { return w_pattern().nz[i][j]; }

// chol6p, fwd6p and bwd6p on the pattern of W
template <typename T>
__host__ __device__ inline void chol6w(T a[21]) {
#pragma unroll
    for (int jj = 0; jj < 6; ++jj) {
        T d = a[tri6(jj, jj)];
#pragma unroll
        for (int k = 0; k < jj; ++k)
            if (wnz(jj, k)) d -= a[tri6(jj, k)] * a[tri6(jj, k)];
        const T inv = (T)1 / sqrt(d);
        a[tri6(jj, jj)] = inv;
#pragma unroll
        for (int ii = jj + 1; ii < 6; ++ii) {
            if (!wnz(ii, jj)) continue;
            T s = a[tri6(ii, jj)];
#pragma unroll
            for (int k = 0; k < jj; ++k)
                if (wnz(ii, k) && wnz(jj, k)) s -= a[tri6(ii, k)] * a[tri6(jj, k)];
            a[tri6(ii, jj)] = s * inv;
        }
    }
}

template <typename T>
__host__ __device__ inline void fwd6w(const T l[21], T v[6]) {
#pragma unroll
    for (int ii = 0; ii < 6; ++ii) {
        T s = v[ii];
#pragma unroll
        for (int k = 0; k < ii; ++k)
            if (wnz(ii, k)) s -= l[tri6(ii, k)] * v[k];
        v[ii] = s * l[tri6(ii, ii)];
    }
}

template <typename T>
__host__ __device__ inline void bwd6w(const T l[21], T v[6]) {
#pragma unroll
    for (int ii = 5; ii >= 0; --ii) {
        T s = v[ii];
#pragma unroll
        for (int k = ii + 1; k < 6; ++k)
            if (wnz(k, ii)) s -= l[tri6(k, ii)] * v[k];
        v[ii] = s * l[tri6(ii, ii)];
    }
}

// W: RT0 mass on the six star edges, star triangle k holding the edge pair star_wpair(k, .),
// unit diagonal on absent edges; factored in place
template <typename T, bool ALLP = false, typename KV>
__host__ __device__ inline void star_w_factor(const DevPatchClass<T>& pc, const KV& kv, const T* __restrict__ wblk,
                                              T w[21]) {
#pragma unroll
    for (int q = 0; q < 21; ++q) w[q] = 0;
#pragma unroll
    for (int kq = 0; kq < 6; ++kq)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q <= p; ++q) {
                const int a = star_wpair(kq, p), b = star_wpair(kq, q);
                if (ALLP || (pc.present[8 + a] && pc.present[8 + b])) w[tri6(a, b)] += wblk[(kq * 2 + p) * 2 + q] * kv_at<T>(kv, kq);
            }
#pragma unroll
    for (int a = 0; a < 6; ++a)
        if (!ALLP && !pc.present[8 + a]) w[tri6(a, a)] = 1;
    chol6w(w);
}

// The residual-independent part of a patch solve, which depends on the permeability only:
// w = L_W (Cholesky factor of the star's RT0 mass W, 1 / L_jj on the diagonal) and s = the
// Cholesky factor of S = C + G + Q W^-1 Q^T with the rank-one shift on the star-constant
// direction (see patch_apply).  Both the factorization and the relaxation step apply
// W^-1 = L_W^-T L_W^-1 and read Q from the class data, so that only w, s and one 6-vector are
// live (42 values per patch, stored by k_patch_factors on the small levels).
constexpr int PFAC = 21 + 21;
template <typename T>
struct PatchFac {
    T w[21];
    T s[21];
};

static_assert(sizeof(PatchFac<double>) == PFAC * sizeof(double), "factor record layout");

template <typename T, bool ALLP = false, typename KV>
__host__ __device__ inline void patch_factor(const DevPatchClass<T>& pc, const KV& kv, const T* __restrict__ wblk,
                                             PatchFac<T>& f) {
    star_w_factor<T, ALLP>(pc, kv, wblk, f.w);
    BIOT_PHASE_FENCE();
    // S = C + G + Q W^-1 Q^T one column at a time (y = W^-1 (row q2 of Q)^T), so that only one
    // 6-vector is live besides the two factors; then the shift beta (1 1^T on the present
    // pressures), beta = tr(S) / k^2
#pragma unroll
    for (int q2 = 0; q2 < 6; ++q2) {
        T y[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) y[a] = pc.Q[q2][a];
        fwd6w(f.w, y);
        bwd6w(f.w, y);
#pragma unroll
        for (int q1 = q2; q1 < 6; ++q1) {
            T v = pc.G[q1][q2];
#pragma unroll
            for (int a = 0; a < 6; ++a) v += pc.Q[q1][a] * y[a];
            f.s[tri6(q1, q2)] = v;
        }
        BIOT_PHASE_FENCE();
    }
    int k = 0;
    T tr = 0;
#pragma unroll
    for (int q1 = 0; q1 < 6; ++q1) {
        f.s[tri6(q1, q1)] += pc.c[q1];
        if (ALLP || pc.present[14 + q1]) {
            ++k;
            tr += f.s[tri6(q1, q1)];
        }
    }
    const T rk = (T)1 / (T)k;
    const T beta = tr * rk * rk;
#pragma unroll
    for (int q1 = 0; q1 < 6; ++q1)
#pragma unroll
        for (int q2 = 0; q2 <= q1; ++q2) {
            if (ALLP || (pc.present[14 + q1] && pc.present[14 + q2]))
                f.s[tri6(q1, q2)] += beta;
            else
                f.s[tri6(q1, q2)] = (q1 == q2) ? (T)1 : (T)0;
        }
    chol6p(f.s);
}

// rr(s): the patch residual at slot s (absent slots hold 0), read where each phase needs it (an
// array, or the staged residual in LDS, so that it need not stay in registers); f: the patch's
// factors (patch_factor); out[a * ostride], a = 0..19, of any type O the values convert to (the
// caller's registers, or the corrections in LDS).  with_mean = false omits the star-mean
// pressure term (the deflated solve).  ALLP: every slot of the patch is present (interior
// class), known at compile time.
// With W = L L^T: Q W^-1 r_w = Q y for y = L^-T L^-1 r_w, and x_w = L^-T L^-1 (r_w - Q^T x_p):
// four substitutions with L, none with a division, and Q read from the class data.
template <typename T, bool ALLP = false, typename RR, typename O>
__host__ __device__ inline void patch_apply(RR&& rr, const DevPatchClass<T>& pc, const PatchFac<T>& f, O* out,
                                            int ostride, bool with_mean = true) {
    T y[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) y[a] = rr(8 + a);
    fwd6w(f.w, y);
    bwd6w(f.w, y);
    BIOT_PHASE_FENCE();
    // rhs = H^T r_u + Q W^-1 r_w - r_p
    T rhs[6];
#pragma unroll
    for (int q1 = 0; q1 < 6; ++q1) {
        T v = -rr(14 + q1);
#pragma unroll
        for (int a = 0; a < 8; ++a) v += pc.H[a][q1] * rr(a);
#pragma unroll
        for (int a = 0; a < 6; ++a) v += pc.Q[q1][a] * y[a];
        rhs[q1] = v;
    }
    // star-mean pressure in closed form; the shifted system (factored in f.s) for the rest
    int k = 0;
    T sum_rp = 0, csum = 0, mrhs = 0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (ALLP || pc.present[14 + q]) {
            ++k;
            sum_rp += rr(14 + q);
            csum += pc.c[q];
            mrhs += rhs[q];
        }
    const T gamma = -sum_rp / csum;
    mrhs *= (T)1 / (T)k;
#pragma unroll
    for (int q1 = 0; q1 < 6; ++q1) rhs[q1] = (ALLP || pc.present[14 + q1]) ? rhs[q1] - mrhs : (T)0;
    BIOT_PHASE_FENCE();
    fwd6p(f.s, rhs);
    bwd6p(f.s, rhs);
    BIOT_PHASE_FENCE();
    // x_p = xp0 + gamma on the present pressures.  The star constant carries no flux
    // (Bh^T 1 = Q^T 1 = 0), so the back-substitutions take the deflated part xp0 alone: the
    // same values in exact arithmetic, without cancelling the often large gamma in rounding.
    T xp[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) xp[q] = (ALLP || pc.present[14 + q]) ? rhs[q] : (T)0;
    // x_u = A^-1 r_u - H x_p
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        T v = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) v += pc.Ainv[a][b] * rr(b);
#pragma unroll
        for (int q = 0; q < 6; ++q) v -= pc.H[a][q] * xp[q];
        out[a * ostride] = (O)((ALLP || pc.present[a]) ? v : (T)0);
    }
    BIOT_PHASE_FENCE();
    // x_w = W^-1 (r_w - Q^T x_p)
    T xw[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        T v = rr(8 + a);
#pragma unroll
        for (int q = 0; q < 6; ++q) v -= pc.Q[q][a] * xp[q];
        xw[a] = v;
    }
    fwd6w(f.w, xw);
    bwd6w(f.w, xw);
#pragma unroll
    for (int a = 0; a < 6; ++a) out[(8 + a) * ostride] = (O)((ALLP || pc.present[8 + a]) ? xw[a] : (T)0);
#pragma unroll
    for (int q = 0; q < 6; ++q)
        out[(14 + q) * ostride] = (O)((ALLP || pc.present[14 + q]) ? xp[q] + (with_mean ? gamma : (T)0) : (T)0);
}

// rr: patch residual (absent slots hold 0); kv: 1/K of the six star triangles;
// wblk: RT0 mass blocks of the star triangles (1/K = 1); out[a * ostride], a = 0..19:
// the factors of the patch formed on the spot, then applied.
template <typename T, bool ALLP = false>
__host__ __device__ inline void patch_solve(const T rr[PATCH], const DevPatchClass<T>& pc, const T kv[6],
                                            const T* __restrict__ wblk, T* out, int ostride,
                                            bool with_mean = true) {
    PatchFac<T> f;
    patch_factor<T, ALLP>(pc, kv, wblk, f);
    patch_apply<T, ALLP>([&](int s) { return rr[s]; }, pc, f, out, ostride, with_mean);
}

}  // namespace biot
