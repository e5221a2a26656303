// Inexact Braess-Sarazin relaxation (Sec. 3.2.2, Appendix D) in two fused launches.
#include "tile.h"
#include "patch_solve.h"

#include <hip/hip_runtime.h>

namespace biot {

// =========================================================================================
// inexact Braess-Sarazin relaxation (Sec. 3.2.2, Appendix D)
// =========================================================================================
// One step on the residual r:
//   z_u = F_u^{-1} r_u            (additive Vanka on the displacement block, 8-DoF patches)
//   z_w = r_w / (tau D_w)         (D_w = diag M_w(K))
//   dp  = omega_J (A_pu z_u + A_pw z_w - r_p) / diag(S)
//   du  = F_u^{-1} (r_u - A_up dp),  dw = (r_w - A_wp dp) / (tau D_w)
//   x  += omega (du, dw, dp)
// with diag(S)_T = (1/M + alpha^2 / (lambda + mu)) |T| + sum_e (tau B_w)_{Te}^2 / (tau D_w)_e.
// Two launches: k_bsr_first (residual, z_u, z_w), k_bsr_second (dp on its window, update).


constexpr int BSR_W = 0;   // planes 0..2 of the diagonal data: 1 / (tau D_w) of w_H, w_V, w_D
constexpr int BSR_S = 3;   // planes 3..4: 1 / diag(S) of p_L, p_U

// diagonal of the RT0 block: the entries of a w row on its own slot
template <typename T>
__global__ __launch_bounds__(256) void k_bsr_wdiag(const T* __restrict__ kinv, const T* __restrict__ coef,
                                                   Layout L, T* __restrict__ d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const long long s = slot_index(L, i, j);
    static_for(std::integer_sequence<int, T_WH, T_WV, T_WD>{}, [&](auto tc) {
        constexpr int t = decltype(tc)::value;
        T v = 0;
        static_for(std::make_integer_sequence<int, SST.n[t]>{}, [&](auto ec) {
            constexpr SEnt en = SST.e[t][decltype(ec)::value];
            if constexpr (en.in == t && en.di == 0 && en.dj == 0) {
                T cc = coef[SST.off[t] + decltype(ec)::value];
                if constexpr (en.kt >= 0) cc *= kinv[en.kt * L.plane + s + (long long)en.kdj * L.pitch + en.kdi];
                v += cc;
            }
        });
        d[(BSR_W + t - T_WH) * L.plane + s] = dof_free(t, i, j, L.n) ? (T)1 / v : (T)0;
    });
}

// diag(S) of the P0 rows from the RT0 diagonal (k_bsr_wdiag first)
template <typename T>
__global__ __launch_bounds__(256) void k_bsr_sdiag(const T* __restrict__ coef, Layout L, T cS,
                                                   T* __restrict__ d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const long long s = slot_index(L, i, j);
    static_for(std::integer_sequence<int, T_PL, T_PU>{}, [&](auto tc) {
        constexpr int t = decltype(tc)::value;
        T v = cS;
        static_for(std::make_integer_sequence<int, SST.n[t]>{}, [&](auto ec) {
            constexpr SEnt en = SST.e[t][decltype(ec)::value];
            if constexpr (tfield(en.in) == 1) {
                static_assert(en.kt < 0, "B_w does not depend on K");
                const T cc = coef[SST.off[t] + decltype(ec)::value];
                // column slots s + (0..1, 0..1) lie inside the padded plane
                v += cc * cc * d[(BSR_W + en.in - T_WH) * L.plane + s + (long long)en.dj * L.pitch + en.di];
            }
        });
        d[(BSR_S + t - T_PL) * L.plane + s] = dof_free(t, i, j, L.n) ? (T)1 / v : (T)0;
    });
}

template <typename T>
void launch_bsr_diag(const LevelView<T>& lv, T cS, T* d, hipStream_t st) {
    dim3 blk(64, 4);
    dim3 grd((lv.L.n + 1 + 63) / 64, (lv.L.n + 1 + 3) / 4);
    hipLaunchKernelGGL(k_bsr_wdiag<T>, grd, blk, 0, st, lv.kinv, lv.coef, lv.L, d);
    hipLaunchKernelGGL(k_bsr_sdiag<T>, grd, blk, 0, st, lv.coef, lv.L, cS, d);
}
template void launch_bsr_diag<double>(const LevelView<double>&, double, double*, hipStream_t);
template void launch_bsr_diag<float>(const LevelView<float>&, float, float*, hipStream_t);

constexpr int NU = 5;   // displacement DoF types ux, uy, bH, bV, bD

// Tiles as in the Vanka step: 16 x 16 threads, VT x VT vertices from (i0, j0), VO x VO owned
// slots; one residual slot of (i0-1 .. i0+VT-1)^2 per thread.

// displacement-patch solves (8 x 8 class inverses, identity on absent DoFs) of the tile's
// vertices from the displacement residual ru (slots i0-1 .. i0+VT-1): so[a][ty][tx]
// With NZ thread layers, layer tz forms the outputs a = tz * 8 / NZ .. (tz + 1) * 8 / NZ - 1.
template <typename T, int NZ>
__device__ __forceinline__ void upatch_solves(const T (&ru)[NU][RW][RW], const T (&ui)[9][64], T (&so)[8][VT][VT],
                                              int i0, int j0, int n, int tx, int ty, int tz) {
    constexpr int NA = 8 / NZ;
    if (tx >= VT || ty >= VT) return;
    const int vi = i0 + tx, vj = j0 + ty;
    T out[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) out[a] = 0;
    if (vi <= n && vj <= n) {
        const int ci = vi == 0 ? 0 : (vi == n ? 2 : 1);
        const int cj = vj == 0 ? 0 : (vj == n ? 2 : 1);
        const T* M = ui[3 * cj + ci];
        T rr[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            int t, di, dj;
            patch_slot(a, t, di, dj);
            rr[a] = ru[t][ty + 1 + dj][tx + 1 + di];
        }
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            T v = 0;
#pragma unroll
            for (int b2 = 0; b2 < 8; ++b2) v += M[(tz * NA + a) * 8 + b2] * rr[b2];
            out[a] = v;
        }
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) so[tz * NA + a][ty][tx] = out[a];
}

// weighted sum of the patch corrections at owned slot (tx, ty): P1 in one patch, bubbles in
// the two patches of their end points (weight 1/2)
template <typename T>
__device__ __forceinline__ void upatch_gather(const T (&so)[8][VT][VT], int tx, int ty, T (&du)[NU]) {
    du[T_UX] = so[0][ty][tx];
    du[T_UY] = so[1][ty][tx];
    du[T_BH] = (T)0.5 * (so[3][ty][tx] + so[2][ty][tx + 1]);
    du[T_BV] = (T)0.5 * (so[5][ty][tx] + so[4][ty + 1][tx]);
    du[T_BD] = (T)0.5 * (so[6][ty][tx + 1] + so[7][ty + 1][tx]);
}

template <typename T, int NTH>
__device__ __forceinline__ void load_uinv(const T* __restrict__ uinv, T (&ui)[9][64], int tid) {
    constexpr int NIT = (9 * 64 + NTH - 1) / NTH;
    T v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int q = tid + it * NTH;
        v[it] = q < 9 * 64 ? uinv[q] : (T)0;
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int q = tid + it * NTH;
        if (q < 9 * 64) (&ui[0][0])[q] = v[it];
    }
}

// layer of a displacement type in the displacement residual of the second half
__host__ __device__ constexpr int ugroup(int t, int NZ) { return NZ == 1 ? 0 : (t <= T_UY ? 0 : 1); }

template <typename T, bool UNIFORM, bool PROL>
struct BsrFirstLds {
    T xs[NTYPES][XS][XS];
    T rs[NTYPES][RW][RW];
    T so[8][VT][VT];
    T ui[9][64];
    T ks[UNIFORM ? 1 : 2][UNIFORM ? 1 : KW][UNIFORM ? 1 : KW];
    T xcs[PROL ? NTYPES : 1][PROL ? PCW : 1][PROL ? PCW : 1];
    T cf[NSTENCIL];
    T pwl[PROL ? NPWEIGHTS : 1];
};

// First half of a BSR step: r = b - A x (x: x_in, or x_in + P x_c with PROL, or 0 with ZERO),
// t_u = F_u^{-1} r_u, t_w = r_w / (tau D_w).  Writes r and t on the owned slots, and with PROL
// the prolongated iterate to x_pro (neighbouring tiles still read x_in on their halo).
template <typename T, bool UNIFORM, bool ZERO, bool PROL, int NZ>
__device__ __forceinline__ void bsr_first_tile(const T* __restrict__ x_in, T* __restrict__ x_pro,
                                               const T* __restrict__ b, T* __restrict__ r, T* __restrict__ t,
                                               const Layout& L, const T* __restrict__ kinv, T kinv_s,
                                               const T* __restrict__ coef, const T* __restrict__ uinv,
                                               const T* __restrict__ d, const T* __restrict__ xc, const Layout& Lc,
                                               const T* __restrict__ pw, int bx, int by,
                                               BsrFirstLds<T, UNIFORM, PROL>& sh) {
    static_assert(!(PROL && ZERO), "the prolongation needs an iterate");
    constexpr int NTH = TPB * NZ;
    const int tx = threadIdx.x, ty = threadIdx.y, tz = NZ > 1 ? (int)threadIdx.z : 0;
    const int tid = (tz * TB + ty) * TB + tx;
    const int i0 = bx * VO, j0 = by * VO;
    const int n = L.n;
    {
        Window<T, NTYPES, RW, NTH> wb;
        wb.load(b, L.plane, L, i0 - 1, j0 - 1, tid);
        Window<T, NTYPES, XS, NTH> wx;
        if constexpr (!ZERO) wx.load(x_in, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, 2, KW, NTH> wk;
        if constexpr (!UNIFORM && !ZERO) wk.load(kinv, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, NTYPES, PCW, NTH> wc;
        if constexpr (PROL) wc.load(xc, Lc.plane, Lc, i0 / 2 - 1, j0 / 2 - 1, tid);
        Table<T, NSTENCIL> tcf;
        if constexpr (!ZERO) tcf.load(coef, tid);
        Table<T, NPWEIGHTS> tpw;
        if constexpr (PROL) tpw.load(pw, tid);
        load_uinv<T, NTH>(uinv, sh.ui, tid);
        if constexpr (!ZERO) tcf.store(sh.cf, tid);
        if constexpr (PROL) tpw.store(sh.pwl, tid);
        wb.store(&sh.rs[0][0][0], tid);
        if constexpr (!ZERO) wx.store(&sh.xs[0][0][0], tid);
        if constexpr (!UNIFORM && !ZERO) wk.store(&sh.ks[0][0][0], tid);
        if constexpr (PROL) wc.store(&sh.xcs[0][0][0], tid);
    }
    __syncthreads();
    if constexpr (PROL) {
        prolong_window<T, NTH>(sh.xs, sh.xcs, sh.pwl, i0, j0, n, tid);
        __syncthreads();
    }
    if constexpr (!ZERO) {
        const int si = i0 - 1 + tx, sj = j0 - 1 + ty;
        const bool in = si <= n + 1 && sj <= n + 1;
        T rv[NTYPES];
        static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tcn) {
            constexpr int tt = decltype(tcn)::value;
            if (rgroup(tt, NZ) != tz) return;      // uniform over the wave
            T acc = 0;
            static_for(std::make_integer_sequence<int, SST.n[tt]>{}, [&](auto ec) {
                constexpr int e = decltype(ec)::value;
                constexpr SEnt en = SST.e[tt][e];
                T cc = sh.cf[SST.off[tt] + e];
                if constexpr (en.kt >= 0) {
                    if constexpr (UNIFORM)
                        cc *= kinv_s;
                    else
                        cc *= sh.ks[en.kt][ty + 1 + en.kdj][tx + 1 + en.kdi];
                }
                acc += cc * sh.xs[en.in][ty + 1 + en.dj][tx + 1 + en.di];
            });
            rv[tt] = (in && dof_free(tt, si, sj, n)) ? sh.rs[tt][ty][tx] - acc : (T)0;
        });
        static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tcn) {
            constexpr int tt = decltype(tcn)::value;
            if (rgroup(tt, NZ) == tz) sh.rs[tt][ty][tx] = rv[tt];
        });
        __syncthreads();
    }
    upatch_solves<T, NZ>(reinterpret_cast<const T(&)[NU][RW][RW]>(sh.rs), sh.ui, sh.so, i0, j0, n, tx, ty, tz);
    __syncthreads();
    if (tx < VO && ty < VO) {
        const int si = i0 + tx, sj = j0 + ty;
        if (si <= n && sj <= n) {
            const long long s0 = slot_index(L, si, sj);
            if (ggroup(T_BD, NZ) == tz) {          // displacement types
                T du[NU];
                upatch_gather<T>(sh.so, tx, ty, du);
#pragma unroll
                for (int q = 0; q < NU; ++q) t[q * L.plane + s0] = dof_free(q, si, sj, n) ? du[q] : (T)0;
            }
            if (ggroup(T_WH, NZ) == tz) {          // Darcy types
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    t[(T_WH + q) * L.plane + s0] = sh.rs[T_WH + q][ty + 1][tx + 1] * d[(BSR_W + q) * L.plane + s0];
            }
            static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if (ggroup(q, NZ) != tz) return;
                r[q * L.plane + s0] = sh.rs[q][ty + 1][tx + 1];
                if constexpr (PROL)
                    if (dof_free(q, si, sj, n)) x_pro[q * L.plane + s0] = sh.xs[q][ty + 2][tx + 2];
            });
        }
    }
}

template <typename T, bool UNIFORM, bool ZERO, bool PROL, int NZ>
__global__ __launch_bounds__(TPB * NZ, 2 * NZ) void k_bsr_first(const T* __restrict__ x_in, T* __restrict__ x_pro,
                                                   const T* __restrict__ b,
                                                   T* __restrict__ r, T* __restrict__ t, Layout L,
                                                   const T* __restrict__ kinv, T kinv_s,
                                                   const T* __restrict__ coef, const T* __restrict__ uinv,
                                                   const T* __restrict__ d, const T* __restrict__ xc, Layout Lc,
                                                   const T* __restrict__ pw) {
    __shared__ BsrFirstLds<T, UNIFORM, PROL> sh;
    int bx, by;
    xcd_tile(bx, by);
    bsr_first_tile<T, UNIFORM, ZERO, PROL, NZ>(x_in, x_pro, b, r, t, L, kinv, kinv_s, coef, uinv, d, xc, Lc, pw, bx,
                                               by, sh);
}

// Second half: dp = omega_J (A_pu t_u + A_pw t_w - r_p) / diag(S) on the window the update
// needs, then x_dst = x_src + omega (F_u^{-1}(r_u - A_up dp), (r_w - A_wp dp) / (tau D_w), dp)
// on the owned slots (x_dst may be x_src: each slot is read and written by its own thread).
constexpr int TW = VT + 4;   // staged t: slots i0-2 .. i0+VT+1
constexpr int DW = VT + 3;   // pressure update: slots i0-2 .. i0+VT

template <typename T>
struct BsrSecondLds {
    T ts[8][TW][TW];         // t_u, t_w
    T dp[2][DW][DW];         // r_p, then the pressure update
    T ds[2][DW][DW];         // 1 / diag(S)
    T ru[NU][RW][RW];        // r_u, then r_u - A_up dp
    T so[8][VT][VT];
    T ui[9][64];
    T cf[NSTENCIL];
};

// DPIN: the pressure correction comes from dpin (2 planes, the Schur sweeps below) instead of the
// single weighted-Jacobi step formed here.
template <typename T, bool ZERO, int NZ, bool DPIN>
__device__ __forceinline__ void bsr_second_tile(const T* __restrict__ r, const T* __restrict__ t, const T* x_src,
                                                T* x, const Layout& L, const T* __restrict__ uinv,
                                                const T* __restrict__ coef, const T* __restrict__ d, T omega,
                                                T omega_J, const T* __restrict__ dpin, int bx, int by,
                                                BsrSecondLds<T>& sh) {
    constexpr int NTH = TPB * NZ;
    const int tx = threadIdx.x, ty = threadIdx.y, tz = NZ > 1 ? (int)threadIdx.z : 0;
    const int tid = (tz * TB + ty) * TB + tx;
    const int i0 = bx * VO, j0 = by * VO;
    const int n = L.n;
    {
        Window<T, 8, TW, NTH> wt;
        if constexpr (!DPIN) wt.load(t, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, 2, DW, NTH> wp;
        wp.load(DPIN ? dpin : r + T_PL * L.plane, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, 2, DW, NTH> wd;
        if constexpr (!DPIN) wd.load(d + BSR_S * L.plane, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, NU, RW, NTH> wr;
        wr.load(r, L.plane, L, i0 - 1, j0 - 1, tid);
        Table<T, NSTENCIL> tcf;
        tcf.load(coef, tid);
        load_uinv<T, NTH>(uinv, sh.ui, tid);
        tcf.store(sh.cf, tid);
        if constexpr (!DPIN) wt.store(&sh.ts[0][0][0], tid);
        wp.store(&sh.dp[0][0][0], tid);
        if constexpr (!DPIN) wd.store(&sh.ds[0][0][0], tid);
        wr.store(&sh.ru[0][0][0], tid);
    }
    __syncthreads();
    // pressure update on slots (i0-2 .. i0+VT)^2; its columns reach t at +0 .. +1
    if constexpr (!DPIN)
    for (int q = tid; q < DW * DW; q += NTH) {
        const int bb = q / DW, a = q - bb * DW;
        const int si = i0 - 2 + a, sj = j0 - 2 + bb;
        static_for(std::integer_sequence<int, T_PL, T_PU>{}, [&](auto tc) {
            constexpr int tp = decltype(tc)::value;
            T acc = 0;
            static_for(std::make_integer_sequence<int, SST.n[tp]>{}, [&](auto ec) {
                constexpr int e = decltype(ec)::value;
                constexpr SEnt en = SST.e[tp][e];
                if constexpr (tfield(en.in) != 2) {
                    static_assert(en.kt < 0, "the pressure rows do not depend on K");
                    acc += sh.cf[SST.off[tp] + e] * sh.ts[en.in][bb + en.dj][a + en.di];
                }
            });
            const T v = omega_J * (acc - sh.dp[tp - T_PL][bb][a]) * sh.ds[tp - T_PL][bb][a];
            sh.dp[tp - T_PL][bb][a] = dof_free(tp, si, sj, n) ? v : (T)0;
        });
    }
    __syncthreads();
    // displacement residual after the pressure update, slot (i0-1+tx, j0-1+ty); its pressure
    // columns reach dp at -1 .. 0
    {
        const int si = i0 - 1 + tx, sj = j0 - 1 + ty;
        T rv[NU];
        static_for(std::make_integer_sequence<int, NU>{}, [&](auto tcn) {
            constexpr int tu = decltype(tcn)::value;
            if (ugroup(tu, NZ) != tz) return;      // uniform over the wave
            T acc = 0;
            static_for(std::make_integer_sequence<int, SST.n[tu]>{}, [&](auto ec) {
                constexpr int e = decltype(ec)::value;
                constexpr SEnt en = SST.e[tu][e];
                if constexpr (tfield(en.in) == 2) acc += sh.cf[SST.off[tu] + e] * sh.dp[en.in - T_PL][ty + 1 + en.dj][tx + 1 + en.di];
            });
            rv[tu] = dof_free(tu, si, sj, n) ? sh.ru[tu][ty][tx] - acc : (T)0;
        });
        __syncthreads();
        static_for(std::make_integer_sequence<int, NU>{}, [&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if (ugroup(q, NZ) == tz) sh.ru[q][ty][tx] = rv[q];
        });
    }
    __syncthreads();
    upatch_solves<T, NZ>(sh.ru, sh.ui, sh.so, i0, j0, n, tx, ty, tz);
    __syncthreads();
    if (tx < VO && ty < VO) {
        const int si = i0 + tx, sj = j0 + ty;
        if (si <= n && sj <= n) {
            const long long s0 = slot_index(L, si, sj);
            if (ggroup(T_BD, NZ) == tz) {          // displacement types
                T du[NU];
                upatch_gather<T>(sh.so, tx, ty, du);
#pragma unroll
                for (int q = 0; q < NU; ++q)
                    if (dof_free(q, si, sj, n))
                        x[q * L.plane + s0] = (ZERO ? (T)0 : x_src[q * L.plane + s0]) + omega * du[q];
            }
            if (ggroup(T_PU, NZ) != tz) return;    // the Darcy and pressure types below
            static_for(std::integer_sequence<int, T_WH, T_WV, T_WD>{}, [&](auto tc) {
                constexpr int tw = decltype(tc)::value;
                T acc = 0;
                static_for(std::make_integer_sequence<int, SST.n[tw]>{}, [&](auto ec) {
                    constexpr int e = decltype(ec)::value;
                    constexpr SEnt en = SST.e[tw][e];
                    if constexpr (tfield(en.in) == 2) acc += sh.cf[SST.off[tw] + e] * sh.dp[en.in - T_PL][ty + 2 + en.dj][tx + 2 + en.di];
                });
                const T dwv = (r[tw * L.plane + s0] - acc) * d[(BSR_W + tw - T_WH) * L.plane + s0];
                if (dof_free(tw, si, sj, n)) x[tw * L.plane + s0] = (ZERO ? (T)0 : x_src[tw * L.plane + s0]) + omega * dwv;
            });
#pragma unroll
            for (int q = T_PL; q <= T_PU; ++q)
                if (dof_free(q, si, sj, n))
                    x[q * L.plane + s0] = (ZERO ? (T)0 : x_src[q * L.plane + s0]) + omega * sh.dp[q - T_PL][ty + 2][tx + 2];
        }
    }
}

template <typename T, bool ZERO, int NZ, bool DPIN>
__global__ __launch_bounds__(TPB * NZ, 2 * NZ) void k_bsr_second(const T* __restrict__ r, const T* __restrict__ t,
                                                    const T* x_src, T* x, Layout L, const T* __restrict__ uinv,
                                                    const T* __restrict__ coef, const T* __restrict__ d,
                                                    T omega, T omega_J, const T* __restrict__ dpin) {
    __shared__ BsrSecondLds<T> sh;
    int bx, by;
    xcd_tile(bx, by);
    bsr_second_tile<T, ZERO, NZ, DPIN>(r, t, x_src, x, L, uinv, coef, d, omega, omega_J, dpin, bx, by, sh);
}

// ---- approximate Schur complement sweeps (Sec. 3.2.2, Appendix D) ------------------------------
// S_hat dp = cS dp + sum over the RT0 columns e of a pressure row of A_pw[T,e] (tau D_w)^{-1}_e
// (A_wp dp)_e, cS = (1/M + alpha^2 / (lambda + mu)) |T|.  k_schur_init forms s = (the pressure rows
// of A on the u and w columns) t - r_p on every cell and the first sweep from zero,
// dp = omega_S s / diag(S_hat); k_schur_sweep is one weighted-Jacobi sweep
// dp' = dp + omega_S (s - S_hat dp) / diag(S_hat).  One thread per slot; absent DoFs get 0 (the
// buffers' halo slots are never written and stay 0).  Column offsets stay within one slot, inside
// the padded plane.
template <typename T>
__global__ __launch_bounds__(256) void k_schur_init(const T* __restrict__ r, const T* __restrict__ t,
                                                    const T* __restrict__ coef, const T* __restrict__ d, Layout L,
                                                    T omega_S, T* __restrict__ s_out, T* __restrict__ dp_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const long long s0 = slot_index(L, i, j);
    static_for(std::integer_sequence<int, T_PL, T_PU>{}, [&](auto tc) {
        constexpr int tp = decltype(tc)::value;
        T acc = 0;
        static_for(std::make_integer_sequence<int, SST.n[tp]>{}, [&](auto ec) {
            constexpr int e = decltype(ec)::value;
            constexpr SEnt en = SST.e[tp][e];
            if constexpr (tfield(en.in) != 2)
                acc += coef[SST.off[tp] + e] * t[en.in * L.plane + s0 + (long long)en.dj * L.pitch + en.di];
        });
        const bool f = dof_free(tp, i, j, L.n);
        const T sv = f ? acc - r[tp * L.plane + s0] : (T)0;
        s_out[(tp - T_PL) * L.plane + s0] = sv;
        dp_out[(tp - T_PL) * L.plane + s0] = f ? omega_S * sv * d[(BSR_S + tp - T_PL) * L.plane + s0] : (T)0;
    });
}

template <typename T>
__global__ __launch_bounds__(256) void k_schur_sweep(const T* __restrict__ s_in, const T* __restrict__ dp_in,
                                                     const T* __restrict__ coef, const T* __restrict__ d, Layout L,
                                                     T omega_S, T cS, T* __restrict__ dp_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const long long s0 = slot_index(L, i, j);
    static_for(std::integer_sequence<int, T_PL, T_PU>{}, [&](auto tc) {
        constexpr int tp = decltype(tc)::value;
        if (!dof_free(tp, i, j, L.n)) {
            dp_out[(tp - T_PL) * L.plane + s0] = (T)0;
            return;
        }
        const T dp = dp_in[(tp - T_PL) * L.plane + s0];
        T sd = cS * dp;
        static_for(std::make_integer_sequence<int, SST.n[tp]>{}, [&](auto ec) {
            constexpr int e1 = decltype(ec)::value;
            constexpr SEnt en1 = SST.e[tp][e1];
            if constexpr (tfield(en1.in) == 1) {
                if (dof_free(en1.in, i + en1.di, j + en1.dj, L.n)) {
                    const long long ws = s0 + (long long)en1.dj * L.pitch + en1.di;
                    T g = 0;
                    static_for(std::make_integer_sequence<int, SST.n[en1.in]>{}, [&](auto fc) {
                        constexpr int e2 = decltype(fc)::value;
                        constexpr SEnt en2 = SST.e[en1.in][e2];
                        if constexpr (tfield(en2.in) == 2)
                            g += coef[SST.off[en1.in] + e2] *
                                 dp_in[(en2.in - T_PL) * L.plane + ws + (long long)en2.dj * L.pitch + en2.di];
                    });
                    sd += coef[SST.off[tp] + e1] * g * d[(BSR_W + en1.in - T_WH) * L.plane + ws];
                }
            }
        });
        dp_out[(tp - T_PL) * L.plane + s0] =
            dp + omega_S * (s_in[(tp - T_PL) * L.plane + s0] - sd) * d[(BSR_S + tp - T_PL) * L.plane + s0];
    });
}

// ---- conjugate gradients on the approximate Schur complement (exact BSR in the limit) ------------
// k steps of diag(S_hat)-preconditioned CG on S_hat dp = s from dp = 0, with s as in k_schur_init.
// Every dot product is summed per block (fixed order: a wave butterfly, then the waves in order)
// into red[slot * np + block], and one block of k_cg_scalars adds the np partial sums in a fixed
// order and updates the recurrence's scalars on the device, so no step waits for the host.
// Scalars (double): sc[0] rho = r . z, sc[1] alpha, sc[2] beta.  Vectors: 2 planes each (p_L, p_U).
constexpr int CG_SLOT_RZ = 0, CG_SLOT_PQ = 1;

template <typename T>
__device__ __forceinline__ void cg_block_sum(double v, double* __restrict__ red, int slot, int np) {
    __shared__ double wsum[4];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const double t = wave_sum(v);
    if ((tid & 63) == 0) wsum[tid >> 6] = t;
    __syncthreads();
    if (tid == 0) red[(long long)slot * np + blockIdx.y * gridDim.x + blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// s and the CG start: r = s, z = s / diag(S_hat), p = z, dp = 0; partial sums of r . z
template <typename T>
__global__ __launch_bounds__(256) void k_cg_init(const T* __restrict__ r, const T* __restrict__ t,
                                                 const T* __restrict__ coef, const T* __restrict__ d, Layout L,
                                                 T* __restrict__ cr, T* __restrict__ cz, T* __restrict__ cp,
                                                 T* __restrict__ dp, double* __restrict__ red, int np) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double acc_rz = 0;
    if (i <= L.n && j <= L.n) {
        const long long s0 = slot_index(L, i, j);
        static_for(std::integer_sequence<int, T_PL, T_PU>{}, [&](auto tc) {
            constexpr int tp = decltype(tc)::value;
            T acc = 0;
            static_for(std::make_integer_sequence<int, SST.n[tp]>{}, [&](auto ec) {
                constexpr int e = decltype(ec)::value;
                constexpr SEnt en = SST.e[tp][e];
                if constexpr (tfield(en.in) != 2)
                    acc += coef[SST.off[tp] + e] * t[en.in * L.plane + s0 + (long long)en.dj * L.pitch + en.di];
            });
            const bool f = dof_free(tp, i, j, L.n);
            const T sv = f ? acc - r[tp * L.plane + s0] : (T)0;
            const T zv = f ? sv * d[(BSR_S + tp - T_PL) * L.plane + s0] : (T)0;
            const long long q = (tp - T_PL) * L.plane + s0;
            cr[q] = sv;
            cz[q] = zv;
            cp[q] = zv;
            dp[q] = 0;
            acc_rz += (double)sv * (double)zv;
        });
    }
    cg_block_sum<T>(acc_rz, red, CG_SLOT_RZ, np);
}

// q = S_hat p (as in k_schur_sweep); partial sums of p . q
template <typename T>
__global__ __launch_bounds__(256) void k_cg_apply(const T* __restrict__ cp, const T* __restrict__ coef,
                                                  const T* __restrict__ d, Layout L, T cS, T* __restrict__ cq,
                                                  double* __restrict__ red, int np) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double acc_pq = 0;
    if (i <= L.n && j <= L.n) {
        const long long s0 = slot_index(L, i, j);
        static_for(std::integer_sequence<int, T_PL, T_PU>{}, [&](auto tc) {
            constexpr int tp = decltype(tc)::value;
            const long long q = (tp - T_PL) * L.plane + s0;
            if (!dof_free(tp, i, j, L.n)) {
                cq[q] = (T)0;
                return;
            }
            const T pv = cp[q];
            T sd = cS * pv;
            static_for(std::make_integer_sequence<int, SST.n[tp]>{}, [&](auto ec) {
                constexpr int e1 = decltype(ec)::value;
                constexpr SEnt en1 = SST.e[tp][e1];
                if constexpr (tfield(en1.in) == 1) {
                    if (dof_free(en1.in, i + en1.di, j + en1.dj, L.n)) {
                        const long long ws = s0 + (long long)en1.dj * L.pitch + en1.di;
                        T g = 0;
                        static_for(std::make_integer_sequence<int, SST.n[en1.in]>{}, [&](auto fc) {
                            constexpr int e2 = decltype(fc)::value;
                            constexpr SEnt en2 = SST.e[en1.in][e2];
                            if constexpr (tfield(en2.in) == 2)
                                g += coef[SST.off[en1.in] + e2] *
                                     cp[(en2.in - T_PL) * L.plane + ws + (long long)en2.dj * L.pitch + en2.di];
                        });
                        sd += coef[SST.off[tp] + e1] * g * d[(BSR_W + en1.in - T_WH) * L.plane + ws];
                    }
                }
            });
            cq[q] = sd;
            acc_pq += (double)pv * (double)sd;
        });
    }
    cg_block_sum<T>(acc_pq, red, CG_SLOT_PQ, np);
}

// mode 0: rho = sum of the r . z partials; mode 1: alpha = rho / (p . q) (0 when p . q = 0);
// mode 2: rho' = sum of the r . z partials, beta = rho' / rho (0 when rho = 0), rho = rho'
__global__ __launch_bounds__(256) void k_cg_scalars(const double* __restrict__ red, int np, int mode,
                                                    double* __restrict__ sc) {
    __shared__ double wsum[4];
    const int slot = mode == 1 ? CG_SLOT_PQ : CG_SLOT_RZ;
    double v = 0;
    for (int b = threadIdx.x; b < np; b += blockDim.x) v += red[(long long)slot * np + b];
    const double t = wave_sum(v);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
        if (mode == 0) {
            sc[0] = tot;
        } else if (mode == 1) {
            sc[1] = tot != 0.0 ? sc[0] / tot : 0.0;
        } else {
            sc[2] = sc[0] != 0.0 ? tot / sc[0] : 0.0;
            sc[0] = tot;
        }
    }
}

// dp += alpha p, r -= alpha q, z = r / diag(S_hat); partial sums of r . z
template <typename T>
__global__ __launch_bounds__(256) void k_cg_update(const T* __restrict__ cp, const T* __restrict__ cq,
                                                   const T* __restrict__ d, Layout L, const double* __restrict__ sc,
                                                   T* __restrict__ dp, T* __restrict__ cr, T* __restrict__ cz,
                                                   double* __restrict__ red, int np) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double acc_rz = 0;
    if (i <= L.n && j <= L.n) {
        const T alpha = (T)sc[1];
        const long long s0 = slot_index(L, i, j);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const long long q = k * L.plane + s0;
            if (!dof_free(T_PL + k, i, j, L.n)) continue;
            dp[q] += alpha * cp[q];
            const T rv = cr[q] - alpha * cq[q];
            const T zv = rv * d[(BSR_S + k) * L.plane + s0];
            cr[q] = rv;
            cz[q] = zv;
            acc_rz += (double)rv * (double)zv;
        }
    }
    cg_block_sum<T>(acc_rz, red, CG_SLOT_RZ, np);
}

// p = z + beta p
template <typename T>
__global__ __launch_bounds__(256) void k_cg_direction(const T* __restrict__ cz, Layout L, const double* __restrict__ sc,
                                                      T* __restrict__ cp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const T beta = (T)sc[2];
    const long long s0 = slot_index(L, i, j);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const long long q = k * L.plane + s0;
        if (dof_free(T_PL + k, i, j, L.n)) cp[q] = cz[q] + beta * cp[q];
    }
}

int cg_partials(const Layout& L) {
    return ((L.n + 1 + 63) / 64) * ((L.n + 1 + 3) / 4);
}

template <typename T>
void launch_bsr_step(const LevelView<T>& lv, T* x, const T* b, T* r, T* t, bool x_is_zero, bool uniform, T kinv_s,
                     T omega, T omega_J, const T* xc, const Layout* Lc, const T* pw, T* xtmp, hipStream_t st,
                     const SchurSweeps<T>* sw) {
    constexpr int NZ = 2;   // two thread layers: residual types, patch outputs and updates split
    dim3 blk(TB, TB, NZ);
    dim3 grd((lv.L.n + 1 + VO - 1) / VO, (lv.L.n + 1 + VO - 1) / VO);
    const Layout lc = Lc ? *Lc : lv.L;
    if (xc && (x_is_zero || !xtmp || xtmp == x)) throw ArgError{"the prolongation needs an iterate and a buffer"};
#define BIOT_BSR_FIRST(U, Z, P)                                                                                  \
    hipLaunchKernelGGL((k_bsr_first<T, U, Z, P, NZ>), grd, blk, 0, st, x, xtmp, b, r, t, lv.L, lv.kinv, kinv_s, \
                       lv.coef, lv.uinv, lv.bsrd, xc, lc, pw)
    if (x_is_zero)
        BIOT_BSR_FIRST(true, true, false);
    else if (uniform && xc)
        BIOT_BSR_FIRST(true, false, true);
    else if (uniform)
        BIOT_BSR_FIRST(true, false, false);
    else if (xc)
        BIOT_BSR_FIRST(false, false, true);
    else
        BIOT_BSR_FIRST(false, false, false);
#undef BIOT_BSR_FIRST
    const T* xsrc = xc ? xtmp : x;
    const T* dp = nullptr;
    if (sw && sw->cg > 0) {
        if (!sw->buf || !sw->red) throw ArgError{"Schur CG needs its buffers"};
        // sw->buf: dp, r, z, p, q (2 planes each); sw->red: 2 np partial sums, then 3 scalars
        const long long pl2 = 2 * lv.L.plane;
        T* cdp = sw->buf;
        T* cr = cdp + pl2;
        T* cz = cr + pl2;
        T* cp = cz + pl2;
        T* cq = cp + pl2;
        const int np = cg_partials(lv.L);
        double* red = sw->red;
        double* sc = red + 2 * np;
        dim3 cb(64, 4);
        dim3 cg((lv.L.n + 1 + 63) / 64, (lv.L.n + 1 + 3) / 4);
        hipLaunchKernelGGL(k_cg_init<T>, cg, cb, 0, st, r, t, lv.coef, lv.bsrd, lv.L, cr, cz, cp, cdp, red, np);
        hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, st, red, np, 0, sc);
        for (int k = 0; k < sw->cg; ++k) {
            hipLaunchKernelGGL(k_cg_apply<T>, cg, cb, 0, st, cp, lv.coef, lv.bsrd, lv.L, sw->cS, cq, red, np);
            hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, st, red, np, 1, sc);
            hipLaunchKernelGGL(k_cg_update<T>, cg, cb, 0, st, cp, cq, lv.bsrd, lv.L, sc, cdp, cr, cz, red, np);
            if (k + 1 < sw->cg) {
                hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, st, red, np, 2, sc);
                hipLaunchKernelGGL(k_cg_direction<T>, cg, cb, 0, st, cz, lv.L, sc, cp);
            }
        }
        dp = cdp;
    } else if (sw && sw->sweeps > 1) {
        if (!sw->buf) throw ArgError{"Schur sweeps need their buffer"};
        // sw->buf: s (2 planes), then two pressure buffers of 2 planes each
        T* sv = sw->buf;
        T* pa = sw->buf + 2 * lv.L.plane;
        T* pb = sw->buf + 4 * lv.L.plane;
        dim3 cb(64, 4);
        dim3 cg((lv.L.n + 1 + 63) / 64, (lv.L.n + 1 + 3) / 4);
        hipLaunchKernelGGL(k_schur_init<T>, cg, cb, 0, st, r, t, lv.coef, lv.bsrd, lv.L, sw->omega_S, sv, pa);
        for (int k = 1; k < sw->sweeps; ++k) {
            hipLaunchKernelGGL(k_schur_sweep<T>, cg, cb, 0, st, sv, pa, lv.coef, lv.bsrd, lv.L, sw->omega_S, sw->cS,
                               pb);
            std::swap(pa, pb);
        }
        dp = pa;
    }
#define BIOT_BSR_SECOND(Z, D)                                                                                    \
    hipLaunchKernelGGL((k_bsr_second<T, Z, NZ, D>), grd, blk, 0, st, r, t, xsrc, x, lv.L, lv.uinv, lv.coef,     \
                       lv.bsrd, omega, omega_J, dp)
    if (x_is_zero && dp)
        BIOT_BSR_SECOND(true, true);
    else if (x_is_zero)
        BIOT_BSR_SECOND(true, false);
    else if (dp)
        BIOT_BSR_SECOND(false, true);
    else
        BIOT_BSR_SECOND(false, false);
#undef BIOT_BSR_SECOND
}
template void launch_bsr_step<double>(const LevelView<double>&, double*, const double*, double*, double*, bool, bool,
                                      double, double, double, const double*, const Layout*, const double*, double*,
                                      hipStream_t, const SchurSweeps<double>*);
template void launch_bsr_step<float>(const LevelView<float>&, float*, const float*, float*, float*, bool, bool, float,
                                     float, float, const float*, const Layout*, const float*, float*, hipStream_t,
                                     const SchurSweeps<float>*);

}  // namespace biot
