// Grid transfers (Sec. 3, eq. block_interp; Sec. 3.1): restriction, prolongation, and the
// residual fused with the restriction.
#include "tile.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace biot {

// =========================================================================================
// grid transfers (Sec. 3, 3.1): gather forms of P^T and P
// =========================================================================================
template <typename T, int tc, int e>
__device__ __forceinline__ T rs_term(const T* __restrict__ rf, const Layout& Lf, int I, int J,
                                     const T* __restrict__ w) {
    constexpr RTerm rt = RST.e[tc][e];
    // fine slots 2I + di in [-2, n_f + 1]: inside the padded plane (zero outside the mesh)
    return w[rt.w] * rf[rt.tf * Lf.plane + slot_index(Lf, 2 * I + rt.di, 2 * J + rt.dj)];
}

template <typename T, int tc, int... E>
__device__ __forceinline__ T rs_row(const T* __restrict__ rf, const Layout& Lf, int I, int J,
                                    const T* __restrict__ w, std::integer_sequence<int, E...>) {
    T acc = 0;
    ((acc += rs_term<T, tc, E>(rf, Lf, I, J, w)), ...);
    return acc;
}

template <typename T, int tc>
__device__ __forceinline__ void rs_out(const T* __restrict__ rf, T* __restrict__ rc, const Layout& Lf,
                                       const Layout& Lc, int I, int J, const T* __restrict__ w) {
    const long long o = tc * Lc.plane + slot_index(Lc, I, J);
    const T v = rs_row<T, tc>(rf, Lf, I, J, w, std::make_integer_sequence<int, RST.n[tc]>{});
    rc[o] = dof_free(tc, I, J, Lc.n) ? v : (T)0;
}

template <typename T, int... Ts>
__device__ __forceinline__ void rs_all(const T* __restrict__ rf, T* __restrict__ rc, const Layout& Lf,
                                       const Layout& Lc, int I, int J, const T* __restrict__ w,
                                       std::integer_sequence<int, Ts...>) {
    (rs_out<T, Ts>(rf, rc, Lf, Lc, I, J, w), ...);
}

// r_c = P^T r_f, one thread per coarse slot
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(const T* __restrict__ rf, T* __restrict__ rc, Layout Lf,
                                                  Layout Lc, const T* __restrict__ w) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I > Lc.n || J > Lc.n) return;
    rs_all<T>(rf, rc, Lf, Lc, I, J, w, std::make_integer_sequence<int, NTYPES>{});
}

template <typename T>
void launch_restrict(const Layout& Lf, const Layout& Lc, const T* rf, T* rc, const T* w, hipStream_t st) {
    dim3 blk(64, 4);
    dim3 grd((Lc.n + 1 + 63) / 64, (Lc.n + 1 + 3) / 4);
    hipLaunchKernelGGL(k_restrict<T>, grd, blk, 0, st, rf, rc, Lf, Lc, w);
}
template void launch_restrict<double>(const Layout&, const Layout&, const double*, double*, const double*,
                                      hipStream_t);
template void launch_restrict<float>(const Layout&, const Layout&, const float*, float*, const float*,
                                     hipStream_t);

// r_c = P^T (b - A x) without storing the fine residual.  A block of 16 x 16 threads owns a
// tile of RT x RT coarse slots from (I0, J0); each thread forms the fine residual of one slot
// of the window (2 I0 - 2 .. 2 I0 + 2 RT + 1)^2 that the restriction reads (fine offsets
// -2 .. +1 per coarse slot), from x staged on a one-slot wider window.
constexpr int RT = 7;                // coarse slots per tile side
constexpr int RRW = 2 * RT + 2;      // fine residual window (= 16, one slot per thread)
constexpr int RXW = RRW + 2;         // staged x window
static_assert(RRW == TB, "one fine residual slot per thread");

template <typename T, bool UNIFORM>
struct ResRestrictLds {
    T xs[NTYPES][RXW][RXW];
    T rs[NTYPES][RRW][RRW];
    T ks[UNIFORM ? 1 : 2][UNIFORM ? 1 : RXW][UNIFORM ? 1 : RXW];
    T cf[NSTENCIL];
};

template <typename T, int tc, int e>
__device__ __forceinline__ T rr_term(const T (&rs)[NTYPES][RRW][RRW], int cx, int cy, const T* __restrict__ w) {
    constexpr RTerm rt = RST.e[tc][e];
    return w[rt.w] * rs[rt.tf][2 * cy + 2 + rt.dj][2 * cx + 2 + rt.di];
}

template <typename T, int tc, int... E>
__device__ __forceinline__ T rr_row(const T (&rs)[NTYPES][RRW][RRW], int cx, int cy, const T* __restrict__ w,
                                    std::integer_sequence<int, E...>) {
    T acc = 0;
    ((acc += rr_term<T, tc, E>(rs, cx, cy, w)), ...);
    return acc;
}

template <typename T, bool UNIFORM, int NZ>
__device__ __forceinline__ void residual_restrict_tile(const T* __restrict__ x, const T* __restrict__ b,
                                                       T* __restrict__ rc, const Layout& Lf, const Layout& Lc,
                                                       const T* __restrict__ kinv, T kinv_s,
                                                       const T* __restrict__ coef, const T* __restrict__ w, int bx,
                                                       int by, ResRestrictLds<T, UNIFORM>& sh) {
    constexpr int NTH = TPB * NZ;
    const int tx = threadIdx.x, ty = threadIdx.y, tz = NZ > 1 ? (int)threadIdx.z : 0;
    const int tid = (tz * TB + ty) * TB + tx;
    const int I0 = bx * RT, J0 = by * RT;
    const int f0i = 2 * I0 - 2, f0j = 2 * J0 - 2;   // fine origin of the residual window
    const int n = Lf.n;
    {
        // x on (f0 - 1 .. f0 + RRW)^2; slots below -2 lie outside the padded plane and only
        // feed residuals of slots outside the mesh (masked)
        constexpr int NV = NTYPES * RXW * RXW;
        constexpr int NIT = (NV + NTH - 1) / NTH;
        T v[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * NTH;
            const int p = q / (RXW * RXW), rem = q - p * (RXW * RXW), bj = rem / RXW, ai = rem - bj * RXW;
            const int si = f0i - 1 + ai, sj = f0j - 1 + bj;
            v[it] = (q < NV && si >= -2 && sj >= -2 && si <= n + 1 && sj <= n + 1)
                        ? x[p * Lf.plane + slot_index(Lf, si, sj)] : (T)0;
        }
        T bv[NTYPES];
        const int si = f0i + tx, sj = f0j + ty;
        const bool inb = si >= -2 && sj >= -2 && si <= n + 1 && sj <= n + 1;
#pragma unroll
        for (int t = 0; t < NTYPES; ++t)
            bv[t] = (inb && rgroup(t, NZ) == tz) ? b[t * Lf.plane + slot_index(Lf, si, sj)] : (T)0;
        Table<T, NSTENCIL> tcf;
        tcf.load(coef, tid);
        T kv[UNIFORM ? 1 : (2 * RXW * RXW + NTH - 1) / NTH];
        if constexpr (!UNIFORM) {
#pragma unroll
            for (int it = 0; it < (2 * RXW * RXW + NTH - 1) / NTH; ++it) {
                const int q = tid + it * NTH;
                const int p = q / (RXW * RXW), rem = q - p * (RXW * RXW), bj = rem / RXW, ai = rem - bj * RXW;
                const int ki = f0i - 1 + ai, kj = f0j - 1 + bj;
                kv[it] = (q < 2 * RXW * RXW && ki >= -2 && kj >= -2 && ki <= n + 1 && kj <= n + 1)
                             ? kinv[p * Lf.plane + slot_index(Lf, ki, kj)] : (T)0;
            }
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * NTH;
            if (q < NV) (&sh.xs[0][0][0])[q] = v[it];
        }
#pragma unroll
        for (int t = 0; t < NTYPES; ++t)
            if (rgroup(t, NZ) == tz) sh.rs[t][ty][tx] = bv[t];
        tcf.store(sh.cf, tid);
        if constexpr (!UNIFORM) {
#pragma unroll
            for (int it = 0; it < (2 * RXW * RXW + NTH - 1) / NTH; ++it) {
                const int q = tid + it * NTH;
                if (q < 2 * RXW * RXW) (&sh.ks[0][0][0])[q] = kv[it];
            }
        }
    }
    __syncthreads();
    // fine residual of slot (f0i + tx, f0j + ty), zero on absent DoFs
    {
        const int si = f0i + tx, sj = f0j + ty;
        T rv[NTYPES];
        static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tcn) {
            constexpr int t = decltype(tcn)::value;
            if (rgroup(t, NZ) != tz) return;       // uniform over the wave
            T acc = 0;
            static_for(std::make_integer_sequence<int, SST.n[t]>{}, [&](auto ec) {
                constexpr int e = decltype(ec)::value;
                constexpr SEnt en = SST.e[t][e];
                T cc = sh.cf[SST.off[t] + e];
                if constexpr (en.kt >= 0) {
                    if constexpr (UNIFORM)
                        cc *= kinv_s;
                    else
                        cc *= sh.ks[en.kt][ty + 1 + en.kdj][tx + 1 + en.kdi];
                }
                acc += cc * sh.xs[en.in][ty + 1 + en.dj][tx + 1 + en.di];
            });
            rv[t] = dof_free(t, si, sj, n) ? sh.rs[t][ty][tx] - acc : (T)0;
        });
        static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tcn) {
            constexpr int t = decltype(tcn)::value;
            if (rgroup(t, NZ) == tz) sh.rs[t][ty][tx] = rv[t];
        });
    }
    __syncthreads();
    // restriction of the tile's coarse slots: wave (q / 64) handles one coarse DoF type, so the
    // compile-time restriction row is uniform over the wave
    static_assert(RT * RT <= 64, "one coarse tile per wave");
    for (int q = tid; q < NTYPES * 64; q += NTH) {
        const int tc = q >> 6, slot = q & 63;
        const int cy = slot / RT, cx = slot - cy * RT;
        const int I = I0 + cx, J = J0 + cy;
        if (slot >= RT * RT || I > Lc.n || J > Lc.n) continue;
        T v = 0;
        static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tcn) {
            constexpr int tcc = decltype(tcn)::value;
            if (tcc == tc) v = rr_row<T, tcc>(sh.rs, cx, cy, w, std::make_integer_sequence<int, RST.n[tcc]>{});
        });
        rc[tc * Lc.plane + slot_index(Lc, I, J)] = dof_free(tc, I, J, Lc.n) ? v : (T)0;
    }
}

template <typename T, bool UNIFORM, int NZ>
__global__ __launch_bounds__(TPB * NZ) void k_residual_restrict(const T* __restrict__ x, const T* __restrict__ b,
                                                           T* __restrict__ rc, Layout Lf, Layout Lc,
                                                           const T* __restrict__ kinv, T kinv_s,
                                                           const T* __restrict__ coef, const T* __restrict__ w) {
    __shared__ ResRestrictLds<T, UNIFORM> sh;
    int bx, by;
    xcd_tile(bx, by);
    residual_restrict_tile<T, UNIFORM, NZ>(x, b, rc, Lf, Lc, kinv, kinv_s, coef, w, bx, by, sh);
}

template <typename T>
void launch_residual_restrict(const LevelView<T>& lf, const Layout& Lc, const T* x, const T* b, T* rc,
                              bool uniform, T kinv_s, const T* w, hipStream_t st, const LaunchTiming* tm) {
    constexpr int NZ = 2;   // two thread layers: the residual's types split between them
    dim3 blk(TB, TB, NZ);
    dim3 grd((Lc.n + 1 + RT - 1) / RT, (Lc.n + 1 + RT - 1) / RT);
    hipEvent_t e0 = tm ? tm->start : nullptr, e1 = tm ? tm->stop : nullptr;
    if (uniform)
        hipExtLaunchKernelGGL((k_residual_restrict<T, true, NZ>), grd, blk, 0, st, e0, e1, 0, x, b, rc, lf.L, Lc,
                              lf.kinv, kinv_s, lf.coef, w);
    else
        hipExtLaunchKernelGGL((k_residual_restrict<T, false, NZ>), grd, blk, 0, st, e0, e1, 0, x, b, rc, lf.L, Lc,
                              lf.kinv, kinv_s, lf.coef, w);
}
template void launch_residual_restrict<double>(const LevelView<double>&, const Layout&, const double*,
                                               const double*, double*, bool, double, const double*, hipStream_t,
                                               const LaunchTiming*);
template void launch_residual_restrict<float>(const LevelView<float>&, const Layout&, const float*, const float*,
                                              float*, bool, float, const float*, hipStream_t, const LaunchTiming*);

// fine DoF (tf, parity): sum over the field's coarse local DoFs of its designated triangle;
// xcl[t][dj][di] holds the coarse values of slots (I + di, J + dj), di, dj in {0, 1}
template <typename T, int tf, int pi, int pj, int q>
__device__ __forceinline__ T pr_term(const T (&xcl)[NTYPES][2][2], const T* __restrict__ w) {
    constexpr LDof c = ldof(fine_tri(tf, pi, pj), ffirst(tf) + q);
    return w[widx(tf, pi, pj, q)] * xcl[c.t][c.dj][c.di];
}

template <typename T, int tf, int pi, int pj, int... Q>
__device__ __forceinline__ T pr_row(const T (&xcl)[NTYPES][2][2], const T* __restrict__ w,
                                    std::integer_sequence<int, Q...>) {
    T acc = 0;
    ((acc += pr_term<T, tf, pi, pj, Q>(xcl, w)), ...);
    return acc;
}

template <typename T, int pi, int pj, int tf>
__device__ __forceinline__ void pr_out(const T (&xcl)[NTYPES][2][2], const T (&xfl)[NTYPES][2][2],
                                       T* __restrict__ xf, const Layout& Lf, int I, int J,
                                       const T* __restrict__ w) {
    const int fi = 2 * I + pi, fj = 2 * J + pj;
    const T acc = pr_row<T, tf, pi, pj>(xcl, w, std::make_integer_sequence<int, fcount(tf)>{});
    if (dof_free(tf, fi, fj, Lf.n)) xf[tf * Lf.plane + slot_index(Lf, fi, fj)] = xfl[tf][pj][pi] + acc;
}

template <typename T, int pi, int pj, int... Ts>
__device__ __forceinline__ void pr_all(const T (&xcl)[NTYPES][2][2], const T (&xfl)[NTYPES][2][2],
                                       T* __restrict__ xf, const Layout& Lf, int I, int J,
                                       const T* __restrict__ w, std::integer_sequence<int, Ts...>) {
    (pr_out<T, pi, pj, Ts>(xcl, xfl, xf, Lf, I, J, w), ...);
}

// x_f += P x_c, one thread per coarse slot writing its four fine slots
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(const T* __restrict__ xc, T* __restrict__ xf, Layout Lf,
                                                     Layout Lc, const T* __restrict__ w) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I > Lc.n || J > Lc.n) return;
    T xcl[NTYPES][2][2];
#pragma unroll
    for (int t = 0; t < NTYPES; ++t)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di) xcl[t][dj][di] = xc[t * Lc.plane + slot_index(Lc, I + di, J + dj)];
    // current values of the four fine slots (2I + 1 <= n_f + 1 stays inside the padded plane)
    T xfl[NTYPES][2][2];
#pragma unroll
    for (int t = 0; t < NTYPES; ++t)
#pragma unroll
        for (int pj = 0; pj < 2; ++pj)
#pragma unroll
            for (int pi = 0; pi < 2; ++pi) xfl[t][pj][pi] = xf[t * Lf.plane + slot_index(Lf, 2 * I + pi, 2 * J + pj)];
    constexpr auto seq = std::make_integer_sequence<int, NTYPES>{};
    pr_all<T, 0, 0>(xcl, xfl, xf, Lf, I, J, w, seq);
    pr_all<T, 1, 0>(xcl, xfl, xf, Lf, I, J, w, seq);
    pr_all<T, 0, 1>(xcl, xfl, xf, Lf, I, J, w, seq);
    pr_all<T, 1, 1>(xcl, xfl, xf, Lf, I, J, w, seq);
}

template <typename T>
void launch_prolong_add(const Layout& Lf, const Layout& Lc, const T* xc, T* xf, const T* w, hipStream_t st) {
    dim3 blk(64, 4);
    dim3 grd((Lc.n + 1 + 63) / 64, (Lc.n + 1 + 3) / 4);
    hipLaunchKernelGGL(k_prolong_add<T>, grd, blk, 0, st, xc, xf, Lf, Lc, w);
}
template void launch_prolong_add<double>(const Layout&, const Layout&, const double*, double*, const double*,
                                         hipStream_t);
template void launch_prolong_add<float>(const Layout&, const Layout&, const float*, float*, const float*,
                                        hipStream_t);

}  // namespace biot
