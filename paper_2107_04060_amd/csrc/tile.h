// Tile machinery shared by the fused stencil kernels (additive Vanka step, inexact BSR,
// residual + restriction): compile-time loops, the 16 x 16-thread tile geometry, LDS staging of
// windows and constant tables, the XCD-aware tile numbering, and the prolongation fused into a
// relaxation step (Sec. 3, eq. block_interp).
#pragma once

#include "kernels.h"
#include "structure.h"

#include <type_traits>
#include <utility>

#include <hip/hip_runtime.h>

namespace biot {

// sum over the 64 lanes of a wave (butterfly; every lane gets the same, order-fixed result)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// compile-time loop: f(std::integral_constant<int, T>) for every T of the sequence
template <int... Ts, typename F>
__device__ __forceinline__ void static_for(std::integer_sequence<int, Ts...>, F&& f) {
    (f(std::integral_constant<int, Ts>{}), ...);
}

constexpr int TB = 16;       // threads per block side
constexpr int TPB = TB * TB; // threads per block
constexpr int VT = TB - 1;   // vertices per tile side
constexpr int VO = VT - 1;   // owned slots per tile side
constexpr int XS = VT + 3;   // staged x_in: slots i0-2 .. i0+VT
constexpr int RW = VT + 1;   // residual: slots i0-1 .. i0+VT-1 (one per thread)
constexpr int KW = VT + 2;   // staged 1/K: slots i0-2 .. i0+VT-1
static_assert(RW == TB, "one residual slot per thread");

// Loads of NP planes of a W x W slot window starting at slot (s0i, s0j) (zero outside the
// padded plane), kept in registers so that all loads of a phase are in flight together.
template <typename T, int NP, int W, int NT = TPB>
struct Window {
    static constexpr int NV = NP * W * W;
    static constexpr int NIT = (NV + NT - 1) / NT;
    T v[NIT];
    __device__ __forceinline__ void load(const T* __restrict__ src, long long plane, const Layout& L, int s0i,
                                         int s0j, int tid) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * NT;
            const int p = q / (W * W), rem = q - p * (W * W), bj = rem / W, ai = rem - bj * W;
            const int si = s0i + ai, sj = s0j + bj;
            v[it] = (q < NV && si <= L.n + 1 && sj <= L.n + 1) ? src[p * plane + slot_index(L, si, sj)] : (T)0;
        }
    }
    __device__ __forceinline__ void store(T* dst, int tid) const {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * NT;
            if (q < NV) dst[q] = v[it];
        }
    }
};

// Kernels with NZ thread layers of 16 x 16 split the DoF types of a slot among the layers:
// rgroup(t) is the layer that forms the residual of type t (two layers get about half of the
// 159 stencil entries each), ggroup(t) the layer that writes type t's output.
__host__ __device__ constexpr int rgroup(int t, int NZ) {
    return NZ == 1 ? 0 : ((t == T_UX || t == T_UY || t == T_WH || t == T_WV) ? 0 : 1);
}
__host__ __device__ constexpr int ggroup(int t, int NZ) { return NZ == 1 ? 0 : (t <= T_BD ? 0 : 1); }

// Tile of this block.  The dispatcher deals consecutive block ids to the 8 XCDs in turn; the
// tiles are renumbered so that the blocks one XCD receives cover a contiguous band of tiles,
// whose shared halo cache lines then meet in that XCD's L2.
constexpr int NXCD = 8;
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
    const int nb = gridDim.x * gridDim.y;
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    const int xcd = b % NXCD, k = b / NXCD;
    const int base = nb / NXCD, rem = nb % NXCD;
    const int t = xcd * base + min(xcd, rem) + k;
    by = t / gridDim.x;
    bx = t - by * gridDim.x;
}

// A table of N <= TPB per-level constants (stencil coefficients, transfer weights) staged in
// LDS together with the tile's windows: one vector load per thread, issued with the others.
// Read from LDS (a broadcast), the constants cost no memory round trip inside the compute
// phase, where scalar loads would wait on the scalar cache one batch at a time.
template <typename T, int N>
struct Table {
    static_assert(N <= TPB, "one element per thread (blocks have at least TPB threads)");
    T v;
    __device__ __forceinline__ void load(const T* __restrict__ src, int tid) { v = tid < N ? src[tid] : (T)0; }
    __device__ __forceinline__ void store(T* dst, int tid) const {
        if (tid < N) dst[tid] = v;
    }
};

// (P x_c) at the fine DoF of type tf anchored at fine slot (2 I + pi, 2 J + pj), from the
// coarse values xcs[t][J - Jc0 + .][I - Ic0 + .] (designated coarse triangle, structure.h)
constexpr int PCW = (VT + 3) / 2 + 2;   // staged coarse window of the prolongation (11)

template <typename T, int tf, int pi, int pj>
__device__ __forceinline__ T prolong_value(const T (&xcs)[NTYPES][PCW][PCW], int ci, int cj,
                                           const T* __restrict__ w) {
    T acc = 0;
    static_for(std::make_integer_sequence<int, fcount(tf)>{}, [&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr LDof c = ldof(fine_tri(tf, pi, pj), ffirst(tf) + q);
        acc += w[widx(tf, pi, pj, q)] * xcs[c.t][cj + c.dj][ci + c.di];
    });
    return acc;
}

// x += P x_c on a staged fine window xs (fine slots i0 - 2 .. i0 + VT, free fine DoFs only) from
// the staged coarse window xcs (coarse slots i0/2 - 1 ..).  Work item: one fine slot, all types.
// The NTH threads are dealt to the four parity classes (2 I + pi, 2 J + pj) of the fine slots,
// NTH / 4 to a class, so the parity, and with it the prolongation stencil, is uniform over a
// wave and known at compile time.
template <typename T, int NTH>
__device__ __forceinline__ void prolong_window(T (&xs)[NTYPES][XS][XS], const T (&xcs)[NTYPES][PCW][PCW],
                                               const T* __restrict__ pwl, int i0, int j0, int n, int tid) {
    constexpr int NCW = (XS + 1) / 2;          // coarse slots whose fine slots meet the window
    constexpr int TPC = NTH / 4;               // threads per parity class
    static_assert(TPC % 64 == 0, "one parity class per wave");
    const int pcls = tid / TPC, r0 = tid - pcls * TPC;
    static_for(std::make_integer_sequence<int, 4>{}, [&](auto pc) {
        constexpr int pi = decltype(pc)::value & 1, pj = decltype(pc)::value >> 1;
        if (pcls != decltype(pc)::value) return;   // uniform over the wave
        for (int r = r0; r < NCW * NCW; r += TPC) {
            const int cj = r / NCW, ci = r - cj * NCW;
            const int a = 2 * ci + pi, bb = 2 * cj + pj;   // window index of fine slot (2I+pi, 2J+pj)
            if (a < XS && bb < XS) {
                const int I = i0 / 2 - 1 + ci, J = j0 / 2 - 1 + cj;
                static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tcn) {
                    constexpr int tf = decltype(tcn)::value;
                    if (dof_free(tf, 2 * I + pi, 2 * J + pj, n))
                        xs[tf][bb][a] += prolong_value<T, tf, pi, pj>(xcs, ci, cj, pwl);
                });
            }
        }
    });
}

}  // namespace biot
