// Device kernels of the RQ Biot multigrid for gfx950 (CDNA4, 64-wide wavefronts).
//
// Paper passages: operator -- Sec. 2.1 (block_form), 2.3 (block_form_rq), Appendix A;
// additive Vanka -- Sec. 3.2.1; transfers -- Sec. 3 (eq. block_interp), 3.1; coarse direct
// solve and FGMRES -- Sec. 5.1.
#include "kernels.h"
#include "patch_solve.h"
#include "structure.h"

#include <type_traits>
#include <utility>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace biot {

// compile-time loop: f(std::integral_constant<int, T>) for every T of the sequence
template <int... Ts, typename F>
__device__ __forceinline__ void static_for(std::integer_sequence<int, Ts...>, F&& f) {
    (f(std::integral_constant<int, Ts>{}), ...);
}

// =========================================================================================
// vector plumbing
// =========================================================================================
template <typename T>
__global__ void k_fill(T* __restrict__ x, long long n, T v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) x[i] = v;
}

void launch_fill(double* x, long long n, double v, hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill<double>, dim3(blocks), dim3(256), 0, st, x, n, v);
}
void launch_fill(float* x, long long n, float v, hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(256), 0, st, x, n, v);
}

// canonical index k -> (type, i, j) of the free DoF
__device__ inline void canon_decode(long long k, const Canon& C, int n, int& t, int& i, int& j) {
    t = 0;
#pragma unroll
    for (int q = 1; q < NTYPES; ++q)
        if (k >= C.off[q]) t = q;
    long long r = k - C.off[t];
    if (t == T_UX || t == T_UY) {
        i = (int)(r % (n - 1)) + 1;
        j = (int)(r / (n - 1)) + 1;
    } else if (t == T_BH || t == T_WH) {
        i = (int)(r % n);
        j = (int)(r / n) + 1;
    } else if (t == T_BV || t == T_WV) {
        i = (int)(r % (n - 1)) + 1;
        j = (int)(r / (n - 1));
    } else {
        i = (int)(r % n);
        j = (int)(r / n);
    }
}

__global__ void k_pack(const double* __restrict__ c, double* __restrict__ x, Layout L, Canon C) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= C.off[NTYPES]) return;
    int t, i, j;
    canon_decode(k, C, L.n, t, i, j);
    x[t * L.plane + slot_index(L, i, j)] = c[k];
}

__global__ void k_unpack(const double* __restrict__ x, double* __restrict__ c, Layout L, Canon C) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= C.off[NTYPES]) return;
    int t, i, j;
    canon_decode(k, C, L.n, t, i, j);
    c[k] = x[t * L.plane + slot_index(L, i, j)];
}

void launch_pack(const double* canon, double* padded, const Layout& L, const Canon& C, hipStream_t st) {
    launch_fill(padded, L.len, 0.0, st);
    long long nf = C.off[NTYPES];
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, canon, padded, L, C);
}
void launch_unpack(const double* padded, double* canon, const Layout& L, const Canon& C, hipStream_t st) {
    long long nf = C.off[NTYPES];
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, padded, canon, L, C);
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ s, D* __restrict__ d, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) d[i] = (D)s[i];
}
void launch_convert(const double* src, float* dst, long long n, hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL((k_convert<double, float>), dim3(blocks), dim3(256), 0, st, src, dst, n);
}
void launch_convert(const float* src, double* dst, long long n, hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(blocks), dim3(256), 0, st, src, dst, n);
}

// =========================================================================================
// operator (rediscretized RQ Biot stencil)
// =========================================================================================
// One output row: sum over the compile-time stencil of the row's type.
template <typename T, int t, int e>
__device__ __forceinline__ T st_term(const T* __restrict__ x, const T* __restrict__ kinv, long long s, int pitch,
                                     long long plane, const T* __restrict__ c) {
    constexpr SEnt en = SST.e[t][e];
    T cc = c[SST.off[t] + e];
    if constexpr (en.kt >= 0) cc *= kinv[en.kt * plane + s + (long long)en.kdj * pitch + en.kdi];
    return cc * x[en.in * plane + s + (long long)en.dj * pitch + en.di];
}

template <typename T, int t, int... E>
__device__ __forceinline__ T st_row(const T* __restrict__ x, const T* __restrict__ kinv, long long s, int pitch,
                                    long long plane, const T* __restrict__ c, std::integer_sequence<int, E...>) {
    T acc = 0;
    ((acc += st_term<T, t, E>(x, kinv, s, pitch, plane, c)), ...);
    return acc;
}

template <typename T, int MODE, int t>
__device__ __forceinline__ void st_out(const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y,
                                       const T* __restrict__ kinv, const Layout& L, long long s, int i, int j,
                                       const T* __restrict__ c) {
    // computed for every slot (neighbours stay inside the padded plane), masked on store
    const bool f = dof_free(t, i, j, L.n);
    const long long o = t * L.plane + s;
    const T acc = st_row<T, t>(x, kinv, s, L.pitch, L.plane, c, std::make_integer_sequence<int, SST.n[t]>{});
    const T val = MODE ? b[o] - acc : acc;
    y[o] = f ? val : (T)0;
}

template <typename T, int MODE, int... Ts>
__device__ __forceinline__ void st_all(const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y,
                                       const T* __restrict__ kinv, const Layout& L, long long s, int i, int j,
                                       const T* __restrict__ c, std::integer_sequence<int, Ts...>) {
    (st_out<T, MODE, Ts>(x, b, y, kinv, L, s, i, j, c), ...);
}

// y = A x (MODE 0) or y = b - A x (MODE 1) on slots [0, n]^2; absent DoFs get 0.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_apply(const T* __restrict__ x, const T* __restrict__ b,
                                               T* __restrict__ y, const T* __restrict__ kinv, Layout L,
                                               const T* __restrict__ coef) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const long long s = slot_index(L, i, j);
    st_all<T, MODE>(x, b, y, kinv, L, s, i, j, coef, std::make_integer_sequence<int, NTYPES>{});
}

template <typename T>
void launch_apply(const LevelView<T>& lv, const T* x, const T* b, T* y, int mode, hipStream_t st) {
    dim3 blk(64, 4);
    dim3 grd((lv.L.n + 1 + 63) / 64, (lv.L.n + 1 + 3) / 4);
    if (mode)
        hipLaunchKernelGGL((k_apply<T, 1>), grd, blk, 0, st, x, b, y, lv.kinv, lv.L, lv.coef);
    else
        hipLaunchKernelGGL((k_apply<T, 0>), grd, blk, 0, st, x, b, y, lv.kinv, lv.L, lv.coef);
}
template void launch_apply<double>(const LevelView<double>&, const double*, const double*, double*, int,
                                   hipStream_t);
template void launch_apply<float>(const LevelView<float>&, const float*, const float*, float*, int, hipStream_t);

// =========================================================================================
// additive Vanka (Sec. 3.2.1), fused with the residual
// =========================================================================================
// One step  x_out = x_in + omega sum_l V_l^T D_l A_l^{-1} V_l (b - A x_in)  per launch.  A block
// of 16 x 16 threads handles a tile of VT x VT vertices starting at (i0, j0) and owns the slots
// of its first VO x VO vertices.  Every thread forms the residual of one slot of
// (i0-1 .. i0+VT)^2 from x_in staged in LDS on a two-slot halo; the threads of the VT x VT
// vertices solve their patches; the owned slots gather the weighted corrections.  x_in and
// x_out are different buffers (neighbouring tiles read x_in on the halo).  ZERO: x_in = 0, the
// residual is b and x_in is not read.
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
template <typename T, int NP, int W>
struct Window {
    static constexpr int NV = NP * W * W;
    static constexpr int NIT = (NV + TPB - 1) / TPB;
    T v[NIT];
    __device__ __forceinline__ void load(const T* __restrict__ src, long long plane, const Layout& L, int s0i,
                                         int s0j, int tid) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * TPB;
            const int p = q / (W * W), rem = q - p * (W * W), bj = rem / W, ai = rem - bj * W;
            const int si = s0i + ai, sj = s0j + bj;
            v[it] = (q < NV && si <= L.n + 1 && sj <= L.n + 1) ? src[p * plane + slot_index(L, si, sj)] : (T)0;
        }
    }
    __device__ __forceinline__ void store(T* dst, int tid) const {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * TPB;
            if (q < NV) dst[q] = v[it];
        }
    }
};

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
    static_assert(N <= TPB, "one element per thread");
    T v;
    __device__ __forceinline__ void load(const T* __restrict__ src, int tid) { v = tid < N ? src[tid] : (T)0; }
    __device__ __forceinline__ void store(T* dst, int tid) const {
        if (tid < N) dst[tid] = v;
    }
};

__device__ inline double vanka_weight(int t, int i, int j, int n) {
    if (t <= T_UY) return 1.0;
    if (t <= T_WD) return 0.5;
    if (t == T_PL) return (i == 0 && j == 0) ? 0.5 : 1.0 / 3.0;
    return (i == n - 1 && j == n - 1) ? 0.5 : 1.0 / 3.0;
}

// LDS offset of patch slot s relative to the residual entry of its vertex (rs[0][vj+1][vi+1])
__host__ __device__ constexpr int pslot_off(int s) {
    const int tt[PATCH] = {T_UX, T_UY, T_BH, T_BH, T_BV, T_BV, T_BD, T_BD, T_WH, T_WH,
                           T_WV, T_WV, T_WD, T_WD, T_PL, T_PL, T_PL, T_PU, T_PU, T_PU};
    const int ddi[PATCH] = {0, 0, -1, 0, 0, 0, -1, 0, -1, 0, 0, 0, -1, 0, 0, -1, 0, -1, -1, 0};
    const int ddj[PATCH] = {0, 0, 0, 0, -1, 0, 0, -1, 0, 0, -1, 0, 0, -1, 0, 0, -1, -1, 0, -1};
    return tt[s] * RW * RW + ddj[s] * RW + ddi[s];
}

// Class-inverse application on the matrix cores (FP64 16x16x4 MFMA), one wave per row of
// the tile: out[a][p] = sum_b M[a][b] r[b][p] for the 16 patches p of a row (the patch index
// is the column of the product, the 20 patch slots its reduction index; M padded to 32 rows).
// Lane layouts of the instruction: A[i][k] in lane 16 k + i, B[k][j] in lane 16 k + j, and
// the result D[i][j] in lane 16 (i % 4) + j, element i / 4 (rows l / 16 + 4 v).
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void mfma_class_frag(const double* M, int lane, double (&af)[2][5]) {
    const int i = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int ks = 0; ks < 5; ++ks) {
            const int row = i + 16 * mb, col = kq + 4 * ks;
            af[mb][ks] = row < PATCH ? M[row * PATCH + col] : 0.0;
        }
}

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

// LDS of the fused step.  The staged x_in and the residual are dead once the patch residuals
// are in registers; the patch corrections then reuse their space.
template <typename T, bool UNIFORM, int NCLS, bool PROL>
struct VankaLds {
    union {
        struct {
            T xs[NTYPES][XS][XS];
            T rs[NTYPES][RW][RW];
        } a;
        T so[PATCH][VT][VT];
    } u;
    T ks[UNIFORM ? 1 : 2][UNIFORM ? 1 : KW][UNIFORM ? 1 : KW];   // 1/K of the L, U triangles
    double ms[UNIFORM ? NCLS : 1][UNIFORM ? PATCH * PATCH : 1];  // class inverses of the tile (FP64)
    T xcs[PROL ? NTYPES : 1][PROL ? PCW : 1][PROL ? PCW : 1];   // coarse iterate (prolongation)
    T cf[NSTENCIL];                                              // stencil coefficients
    T pwl[PROL ? NPWEIGHTS : 1];                                 // prolongation weights
};

// PROL: the iterate is x_in + P x_c (prolongation of the coarse-grid correction, Sec. 3),
// formed on the staged window; x_out = x_in + P x_c + omega (...).
// One tile (bx, by) of the step, by the 16 x 16 threads of a block with LDS sh.
template <typename T, bool UNIFORM, bool ZERO, int NCLS, bool PROL>
__device__ __forceinline__ void vanka_step_tile(const T* __restrict__ x_in, const T* __restrict__ b,
                                                T* __restrict__ x_out, const Layout& L, const T* __restrict__ kinv,
                                                T kinv_s, const T* __restrict__ coef,
                                                const DevPatchClass<double>* __restrict__ cls,
                                                const double* __restrict__ wblk, const double* __restrict__ minv,
                                                T omega, const T* __restrict__ xc, const Layout& Lc,
                                                const T* __restrict__ pw, int bx, int by,
                                                VankaLds<T, UNIFORM, NCLS, PROL>& sh) {
    static_assert(!(PROL && ZERO), "the prolongation needs an iterate");
    auto& xs = sh.u.a.xs;
    auto& rs = sh.u.a.rs;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TB + tx;
    const int i0 = bx * VO, j0 = by * VO;
    const int n = L.n;
    // vertex classes of the tile (0 low edge, 1 interior, 2 high edge per direction); their
    // matrices sit in ms[(cj - cjlo) * cw + (ci - cilo)]
    const int cilo = i0 == 0 ? 0 : 1, cihi = (i0 + VT - 1 >= n) ? 2 : 1;
    const int cjlo = j0 == 0 ? 0 : 1, cjhi = (j0 + VT - 1 >= n) ? 2 : 1;
    const int cw = cihi - cilo + 1;
    // ---- staging: b (and x_in, 1/K), class inverses ---------------------------------------------
    {
        // every load of the staging phase is issued before the first LDS store, so the tile
        // waits for one memory latency, not one per class
        constexpr int NM = PATCH * PATCH;
        constexpr int NIT = (NM + TPB - 1) / TPB;
        constexpr int NCL = UNIFORM ? NCLS : 1;
        const int nc = cw * (cjhi - cjlo + 1);
        double mv[NCL][NIT];
        if constexpr (UNIFORM) {
#pragma unroll
            for (int k = 0; k < NCL; ++k) {
                const int cidx = 3 * (cjlo + k / cw) + cilo + k % cw;
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    const int q = tid + it * TPB;
                    mv[k][it] = (k < nc && q < NM) ? minv[cidx * NM + q] : 0.0;
                }
            }
        }
        Window<T, NTYPES, RW> wb;
        wb.load(b, L.plane, L, i0 - 1, j0 - 1, tid);
        Window<T, NTYPES, XS> wx;
        if constexpr (!ZERO) wx.load(x_in, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, 2, KW> wk;
        if constexpr (!UNIFORM) wk.load(kinv, L.plane, L, i0 - 2, j0 - 2, tid);
        // coarse slots i0/2 - 1 .. i0/2 + PCW - 2 feed the fine window i0 - 2 .. i0 + VT + 1
        Window<T, NTYPES, PCW> wc;
        if constexpr (PROL) wc.load(xc, Lc.plane, Lc, i0 / 2 - 1, j0 / 2 - 1, tid);
        Table<T, NSTENCIL> tcf;
        if constexpr (!ZERO) tcf.load(coef, tid);
        Table<T, NPWEIGHTS> tpw;
        if constexpr (PROL) tpw.load(pw, tid);
        if constexpr (!ZERO) tcf.store(sh.cf, tid);
        if constexpr (PROL) tpw.store(sh.pwl, tid);
        if constexpr (UNIFORM) {
#pragma unroll
            for (int k = 0; k < NCL; ++k)
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    const int q = tid + it * TPB;
                    if (k < nc && q < NM) sh.ms[k][q] = mv[k][it];
                }
        }
        wb.store(&rs[0][0][0], tid);
        if constexpr (!ZERO) wx.store(&xs[0][0][0], tid);
        if constexpr (!UNIFORM) wk.store(&sh.ks[0][0][0], tid);
        if constexpr (PROL) wc.store(&sh.xcs[0][0][0], tid);
    }
    __syncthreads();
    if constexpr (PROL) {
        // x += P x_c on the staged window (free fine DoFs only): the thread of coarse window slot
        // (ci, cj) fills its four fine slots (2 I + pi, 2 J + pj), parities known at compile time
        constexpr int NCW = (XS + 1) / 2;        // coarse slots whose fine slots meet the window
        if (tid < NCW * NCW) {
            const int cj = tid / NCW, ci = tid - cj * NCW;
            const int I = i0 / 2 - 1 + ci, J = j0 / 2 - 1 + cj;
            static_for(std::make_integer_sequence<int, 4>{}, [&](auto pc) {
                constexpr int pi = decltype(pc)::value & 1, pj = decltype(pc)::value >> 1;
                const int a = 2 * ci + pi, bb = 2 * cj + pj;   // window index of fine slot (2I+pi, 2J+pj)
                if (a < XS && bb < XS) {
                    static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tcn) {
                        constexpr int tf = decltype(tcn)::value;
                        if (dof_free(tf, 2 * I + pi, 2 * J + pj, n))
                            xs[tf][bb][a] += prolong_value<T, tf, pi, pj>(sh.xcs, ci, cj, sh.pwl);
                    });
                }
            });
        }
        __syncthreads();
    }
    // ---- residual r = b - A x_in of slot (i0-1+tx, j0-1+ty), zero on absent DoFs -----------------
    if constexpr (!ZERO) {
        const int si = i0 - 1 + tx, sj = j0 - 1 + ty;
        const bool in = si <= n + 1 && sj <= n + 1;
        T rv[NTYPES];
        static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
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
                acc += cc * xs[en.in][ty + 1 + en.dj][tx + 1 + en.di];
            });
            rv[t] = (in && dof_free(t, si, sj, n)) ? rs[t][ty][tx] - acc : (T)0;
        });
#pragma unroll
        for (int t = 0; t < NTYPES; ++t) rs[t][ty][tx] = rv[t];
        __syncthreads();
    }
    // ---- patch solves of the tile's vertices ----------------------------------------------------
    const int vi = i0 + tx, vj = j0 + ty;
    const bool patch = tx < VT && ty < VT;
    T xown[NTYPES];
#pragma unroll
    for (int t = 0; t < NTYPES; ++t) xown[t] = (ZERO || !patch) ? (T)0 : xs[t][ty + 2][tx + 2];
    // The patch arithmetic is FP64 for either storage precision T.
    if constexpr (UNIFORM) {
        // The products run over batches of up to 16 patches that share one class inverse: each
        // tile row (its patches at interior-class columns), each boundary column of the tile
        // (its patches at interior-class rows) and each corner patch.  Wave w takes rows
        // w, w + 4, w + 8, w + 12 and the boundary batches dealt to it (the i-th present one goes
        // to wave 3 - i % 4), so a boundary tile costs one product per batch, not one per class
        // present in a row.
        const int lane = tid & 63, wave = tid >> 6;
        const int jl = lane & 15, kq = lane >> 4;
        auto vcls = [n](int v) { return v == 0 ? 0 : (v == n ? 2 : 1); };
        const int bcl = i0 == 0 ? 0 : -1, bcr = n - i0 < VT ? n - i0 : -1;   // tile columns of i = 0, n
        const int brb = j0 == 0 ? 0 : -1, brt = n - j0 < VT ? n - j0 : -1;   // tile rows of j = 0, n
        // boundary batches e in a fixed order: left, right column; corners (l,b), (r,b), (l,t),
        // (r,t): tile column eti(e) and, for corners, tile row etj(e); -1 where the tile does
        // not reach that boundary
        auto eti = [&](int e) { return (e & 1) ? bcr : bcl; };
        auto etj = [&](int e) { return e < 2 ? 0 : (e < 4 ? brb : brt); };
        auto epr = [&](int e) { return eti(e) >= 0 && etj(e) >= 0; };
        // batch slots of this wave: 0..3 rows, 4..5 boundary batches (e index, or -1)
        int ex0 = -1, ex1 = -1;
        {
            int cnt = 0;
#pragma unroll
            for (int e = 0; e < 6; ++e)
                if (epr(e)) {
                    if (cnt == 3 - wave) ex0 = e;
                    if (cnt == 7 - wave) ex1 = e;
                    ++cnt;
                }
        }
        // batch s: active, class (cj, ci), the lane's patch (pti, ptj) and whether it belongs to it
        auto batch = [&](int s, bool& act, int& cj, int& ci, int& pti, int& ptj, bool& own) {
            if (s < 4) {
                ptj = wave + 4 * s;
                pti = jl;
                act = ptj < VT && j0 + ptj <= n;
                cj = act ? vcls(j0 + ptj) : 1;
                ci = 1;
                own = act && pti < VT && i0 + pti <= n && vcls(i0 + pti) == 1;
            } else {
                const int e = s == 4 ? ex0 : ex1;
                act = e >= 0;
                if (e >= 0 && e < 2) {             // boundary column
                    pti = eti(e);
                    ptj = jl;
                    ci = vcls(i0 + pti);
                    cj = 1;
                    own = ptj < VT && j0 + ptj <= n && vcls(j0 + ptj) == 1;
                } else if (e >= 2) {               // corner patch, column 0 of the product
                    pti = eti(e);
                    ptj = etj(e);
                    ci = vcls(i0 + pti);
                    cj = vcls(j0 + ptj);
                    own = jl == 0;
                } else {
                    pti = ptj = 0;
                    ci = cj = 1;
                    own = false;
                }
            }
        };
        // residuals of the batches' patches (B operand), read before the corrections overwrite
        // the residual array; lanes outside a batch read any patch of the tile
        double bf[6][5];
#pragma unroll
        for (int sb = 0; sb < 6; ++sb) {
            bool act, own;
            int cj, ci, pti, ptj;
            batch(sb, act, cj, ci, pti, ptj, own);
            const T* base = &rs[0][0][0] + (min(ptj, VT - 1) + 1) * RW + (min(pti, VT - 1) + 1);
#pragma unroll
            for (int ks = 0; ks < 5; ++ks) {
                const int o = kq == 0 ? pslot_off(4 * ks) : kq == 1 ? pslot_off(4 * ks + 1)
                            : kq == 2 ? pslot_off(4 * ks + 2) : pslot_off(4 * ks + 3);
                bf[sb][ks] = act ? (double)base[o] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int sb = 0; sb < 6; ++sb) {
            bool act, own;
            int cj, ci, pti, ptj;
            batch(sb, act, cj, ci, pti, ptj, own);
            if (!act) continue;                    // uniform over the wave
            double cf[2][5];
            mfma_class_frag(sh.ms[(cj - cjlo) * cw + (ci - cilo)], lane, cf);
            v4d acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < 5; ++ks) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(cf[0][ks], bf[sb][ks], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(cf[1][ks], bf[sb][ks], acc1, 0, 0, 0);
            }
            // rows a = kq + 4 v + 16 mb of the lane's patch
            if (own) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    sh.u.so[kq + 4 * v][ptj][pti] = (T)acc0[v];
                    if (kq + 4 * v + 16 < PATCH) sh.u.so[kq + 4 * v + 16][ptj][pti] = (T)acc1[v];
                }
            }
        }
    } else {
        // per-patch elimination (permeability varies from patch to patch)
        double out[PATCH];
#pragma unroll
        for (int s = 0; s < PATCH; ++s) out[s] = 0;
        if (patch && vi <= n && vj <= n) {
            const int ci = vi == 0 ? 0 : (vi == n ? 2 : 1);
            const int cj = vj == 0 ? 0 : (vj == n ? 2 : 1);
            const DevPatchClass<double>& pc = cls[3 * cj + ci];
            bool keep = false;
#pragma unroll
            for (int s = 0; s < 14; ++s) keep = keep || pc.present[s];
            if (keep) {
                double rr[PATCH];
#pragma unroll
                for (int s = 0; s < PATCH; ++s) {
                    int t, di, dj;
                    patch_slot(s, t, di, dj);
                    rr[s] = (double)rs[t][ty + 1 + dj][tx + 1 + di];
                }
                double kv[6];
#pragma unroll
                for (int kq = 0; kq < 6; ++kq) {
                    int ut, di, dj;
                    star_tri(kq, ut, di, dj);
                    kv[kq] = (double)sh.ks[ut][ty + 2 + dj][tx + 2 + di];
                }
                patch_solve<double>(rr, pc, kv, wblk, out, 1);
            }
        }
        __syncthreads();
        if (patch) {
#pragma unroll
            for (int s = 0; s < PATCH; ++s) sh.u.so[s][ty][tx] = (T)out[s];
        }
    }
    __syncthreads();
    // ---- weighted gather on the owned slots --------------------------------------------------------
    if (tx < VO && ty < VO) {
        const int si = i0 + tx, sj = j0 + ty;
        if (si <= n && sj <= n) {
            const auto& so = sh.u.so;
            T c[NTYPES];
            c[T_UX] = so[0][ty][tx];
            c[T_UY] = so[1][ty][tx];
            c[T_BH] = so[3][ty][tx] + so[2][ty][tx + 1];
            c[T_BV] = so[5][ty][tx] + so[4][ty + 1][tx];
            c[T_BD] = so[6][ty][tx + 1] + so[7][ty + 1][tx];
            c[T_WH] = so[9][ty][tx] + so[8][ty][tx + 1];
            c[T_WV] = so[11][ty][tx] + so[10][ty + 1][tx];
            c[T_WD] = so[12][ty][tx + 1] + so[13][ty + 1][tx];
            c[T_PL] = so[14][ty][tx] + so[15][ty][tx + 1] + so[16][ty + 1][tx];
            c[T_PU] = so[17][ty + 1][tx + 1] + so[18][ty][tx + 1] + so[19][ty + 1][tx];
            const long long s0 = slot_index(L, si, sj);
#pragma unroll
            for (int t = 0; t < NTYPES; ++t)
                if (dof_free(t, si, sj, n))
                    x_out[t * L.plane + s0] = xown[t] + omega * (T)vanka_weight(t, si, sj, n) * c[t];
        }
    }
}

template <typename T, bool UNIFORM, bool ZERO, int NCLS, bool PROL>
__global__ __launch_bounds__(TPB) void k_vanka_step(const T* __restrict__ x_in, const T* __restrict__ b,
                                                    T* __restrict__ x_out, Layout L, const T* __restrict__ kinv,
                                                    T kinv_s, const T* __restrict__ coef,
                                                    const DevPatchClass<double>* __restrict__ cls,
                                                    const double* __restrict__ wblk,
                                                    const double* __restrict__ minv, T omega,
                                                    const T* __restrict__ xc, Layout Lc,
                                                    const T* __restrict__ pw) {
    __shared__ VankaLds<T, UNIFORM, NCLS, PROL> sh;
    int bx, by;
    xcd_tile(bx, by);
    vanka_step_tile<T, UNIFORM, ZERO, NCLS, PROL>(x_in, b, x_out, L, kinv, kinv_s, coef, cls, wblk, minv, omega, xc,
                                                  Lc, pw, bx, by, sh);
}

template <typename T, bool UNIFORM, bool ZERO, bool PROL>
static void launch_vanka_step_t(const LevelView<T>& lv, const T* x_in, const T* b, T* x_out, T kinv_s, T omega,
                                const T* xc, const Layout& Lc, const T* pw, const LaunchTiming* tm, hipStream_t st) {
    dim3 blk(TB, TB);
    dim3 grd((lv.L.n + 1 + VO - 1) / VO, (lv.L.n + 1 + VO - 1) / VO);
    hipEvent_t e0 = tm ? tm->start : nullptr, e1 = tm ? tm->stop : nullptr;
    // a tile spans at most two vertex classes per direction unless it covers the whole mesh
    if (UNIFORM && lv.L.n + 1 <= VT)
        hipExtLaunchKernelGGL((k_vanka_step<T, UNIFORM, ZERO, 9, PROL>), grd, blk, 0, st, e0, e1, 0, x_in, b, x_out,
                              lv.L, lv.kinv, kinv_s, lv.coef, lv.cls, lv.wblk, lv.minv, omega, xc, Lc, pw);
    else
        hipExtLaunchKernelGGL((k_vanka_step<T, UNIFORM, ZERO, 4, PROL>), grd, blk, 0, st, e0, e1, 0, x_in, b, x_out,
                              lv.L, lv.kinv, kinv_s, lv.coef, lv.cls, lv.wblk, lv.minv, omega, xc, Lc, pw);
}

template <typename T>
void launch_vanka_step(const LevelView<T>& lv, const T* x_in, const T* b, T* x_out, bool uniform, T kinv_s,
                       T omega, hipStream_t st, const T* xc, const Layout* Lc, const T* pw, const LaunchTiming* tm) {
    const Layout lc = Lc ? *Lc : lv.L;
    if (xc && !x_in) throw ArgError{"the prolongation needs an iterate"};
    if (uniform) {
        if (xc)
            launch_vanka_step_t<T, true, false, true>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st);
        else if (x_in)
            launch_vanka_step_t<T, true, false, false>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st);
        else
            launch_vanka_step_t<T, true, true, false>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st);
    } else {
        if (xc)
            launch_vanka_step_t<T, false, false, true>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st);
        else if (x_in)
            launch_vanka_step_t<T, false, false, false>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st);
        else
            launch_vanka_step_t<T, false, true, false>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st);
    }
}
template void launch_vanka_step<double>(const LevelView<double>&, const double*, const double*, double*, bool,
                                        double, double, hipStream_t, const double*, const Layout*, const double*,
                                        const LaunchTiming*);
template void launch_vanka_step<float>(const LevelView<float>&, const float*, const float*, float*, bool, float,
                                       float, hipStream_t, const float*, const Layout*, const float*,
                                       const LaunchTiming*);

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
template <typename T>
__device__ __forceinline__ void upatch_solves(const T (&ru)[NU][RW][RW], const T (&ui)[9][64], T (&so)[8][VT][VT],
                                              int i0, int j0, int n, int tx, int ty) {
    if (tx >= VT || ty >= VT) return;
    const int vi = i0 + tx, vj = j0 + ty;
    T out[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) out[a] = 0;
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
        for (int a = 0; a < 8; ++a) {
            T v = 0;
#pragma unroll
            for (int b2 = 0; b2 < 8; ++b2) v += M[a * 8 + b2] * rr[b2];
            out[a] = v;
        }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) so[a][ty][tx] = out[a];
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

template <typename T>
__device__ __forceinline__ void load_uinv(const T* __restrict__ uinv, T (&ui)[9][64], int tid) {
    T v[3];
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        const int q = tid + it * TPB;
        v[it] = q < 9 * 64 ? uinv[q] : (T)0;
    }
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        const int q = tid + it * TPB;
        if (q < 9 * 64) (&ui[0][0])[q] = v[it];
    }
}

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
template <typename T, bool UNIFORM, bool ZERO, bool PROL>
__device__ __forceinline__ void bsr_first_tile(const T* __restrict__ x_in, T* __restrict__ x_pro,
                                               const T* __restrict__ b, T* __restrict__ r, T* __restrict__ t,
                                               const Layout& L, const T* __restrict__ kinv, T kinv_s,
                                               const T* __restrict__ coef, const T* __restrict__ uinv,
                                               const T* __restrict__ d, const T* __restrict__ xc, const Layout& Lc,
                                               const T* __restrict__ pw, int bx, int by,
                                               BsrFirstLds<T, UNIFORM, PROL>& sh) {
    static_assert(!(PROL && ZERO), "the prolongation needs an iterate");
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TB + tx;
    const int i0 = bx * VO, j0 = by * VO;
    const int n = L.n;
    {
        Window<T, NTYPES, RW> wb;
        wb.load(b, L.plane, L, i0 - 1, j0 - 1, tid);
        Window<T, NTYPES, XS> wx;
        if constexpr (!ZERO) wx.load(x_in, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, 2, KW> wk;
        if constexpr (!UNIFORM && !ZERO) wk.load(kinv, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, NTYPES, PCW> wc;
        if constexpr (PROL) wc.load(xc, Lc.plane, Lc, i0 / 2 - 1, j0 / 2 - 1, tid);
        Table<T, NSTENCIL> tcf;
        if constexpr (!ZERO) tcf.load(coef, tid);
        Table<T, NPWEIGHTS> tpw;
        if constexpr (PROL) tpw.load(pw, tid);
        load_uinv(uinv, sh.ui, tid);
        if constexpr (!ZERO) tcf.store(sh.cf, tid);
        if constexpr (PROL) tpw.store(sh.pwl, tid);
        wb.store(&sh.rs[0][0][0], tid);
        if constexpr (!ZERO) wx.store(&sh.xs[0][0][0], tid);
        if constexpr (!UNIFORM && !ZERO) wk.store(&sh.ks[0][0][0], tid);
        if constexpr (PROL) wc.store(&sh.xcs[0][0][0], tid);
    }
    __syncthreads();
    if constexpr (PROL) {
        constexpr int NCW = (XS + 1) / 2;
        if (tid < NCW * NCW) {
            const int cj = tid / NCW, ci = tid - cj * NCW;
            const int I = i0 / 2 - 1 + ci, J = j0 / 2 - 1 + cj;
            static_for(std::make_integer_sequence<int, 4>{}, [&](auto pc) {
                constexpr int pi = decltype(pc)::value & 1, pj = decltype(pc)::value >> 1;
                const int a = 2 * ci + pi, bb = 2 * cj + pj;
                if (a < XS && bb < XS) {
                    static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tcn) {
                        constexpr int tf = decltype(tcn)::value;
                        if (dof_free(tf, 2 * I + pi, 2 * J + pj, n))
                            sh.xs[tf][bb][a] += prolong_value<T, tf, pi, pj>(sh.xcs, ci, cj, sh.pwl);
                    });
                }
            });
        }
        __syncthreads();
    }
    if constexpr (!ZERO) {
        const int si = i0 - 1 + tx, sj = j0 - 1 + ty;
        const bool in = si <= n + 1 && sj <= n + 1;
        T rv[NTYPES];
        static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tcn) {
            constexpr int tt = decltype(tcn)::value;
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
#pragma unroll
        for (int tt = 0; tt < NTYPES; ++tt) sh.rs[tt][ty][tx] = rv[tt];
        __syncthreads();
    }
    upatch_solves<T>(reinterpret_cast<const T(&)[NU][RW][RW]>(sh.rs), sh.ui, sh.so, i0, j0, n, tx, ty);
    __syncthreads();
    if (tx < VO && ty < VO) {
        const int si = i0 + tx, sj = j0 + ty;
        if (si <= n && sj <= n) {
            const long long s0 = slot_index(L, si, sj);
            T du[NU];
            upatch_gather<T>(sh.so, tx, ty, du);
#pragma unroll
            for (int q = 0; q < NU; ++q) t[q * L.plane + s0] = dof_free(q, si, sj, n) ? du[q] : (T)0;
#pragma unroll
            for (int q = 0; q < 3; ++q)
                t[(T_WH + q) * L.plane + s0] = sh.rs[T_WH + q][ty + 1][tx + 1] * d[(BSR_W + q) * L.plane + s0];
#pragma unroll
            for (int q = 0; q < NTYPES; ++q) r[q * L.plane + s0] = sh.rs[q][ty + 1][tx + 1];
            if constexpr (PROL) {
#pragma unroll
                for (int q = 0; q < NTYPES; ++q)
                    if (dof_free(q, si, sj, n)) x_pro[q * L.plane + s0] = sh.xs[q][ty + 2][tx + 2];
            }
        }
    }
}

template <typename T, bool UNIFORM, bool ZERO, bool PROL>
__global__ __launch_bounds__(TPB) void k_bsr_first(const T* __restrict__ x_in, T* __restrict__ x_pro,
                                                   const T* __restrict__ b,
                                                   T* __restrict__ r, T* __restrict__ t, Layout L,
                                                   const T* __restrict__ kinv, T kinv_s,
                                                   const T* __restrict__ coef, const T* __restrict__ uinv,
                                                   const T* __restrict__ d, const T* __restrict__ xc, Layout Lc,
                                                   const T* __restrict__ pw) {
    __shared__ BsrFirstLds<T, UNIFORM, PROL> sh;
    int bx, by;
    xcd_tile(bx, by);
    bsr_first_tile<T, UNIFORM, ZERO, PROL>(x_in, x_pro, b, r, t, L, kinv, kinv_s, coef, uinv, d, xc, Lc, pw, bx, by,
                                           sh);
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

template <typename T, bool ZERO>
__device__ __forceinline__ void bsr_second_tile(const T* __restrict__ r, const T* __restrict__ t, const T* x_src,
                                                T* x, const Layout& L, const T* __restrict__ uinv,
                                                const T* __restrict__ coef, const T* __restrict__ d, T omega,
                                                T omega_J, int bx, int by, BsrSecondLds<T>& sh) {
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TB + tx;
    const int i0 = bx * VO, j0 = by * VO;
    const int n = L.n;
    {
        Window<T, 8, TW> wt;
        wt.load(t, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, 2, DW> wp;
        wp.load(r + T_PL * L.plane, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, 2, DW> wd;
        wd.load(d + BSR_S * L.plane, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, NU, RW> wr;
        wr.load(r, L.plane, L, i0 - 1, j0 - 1, tid);
        Table<T, NSTENCIL> tcf;
        tcf.load(coef, tid);
        load_uinv(uinv, sh.ui, tid);
        tcf.store(sh.cf, tid);
        wt.store(&sh.ts[0][0][0], tid);
        wp.store(&sh.dp[0][0][0], tid);
        wd.store(&sh.ds[0][0][0], tid);
        wr.store(&sh.ru[0][0][0], tid);
    }
    __syncthreads();
    // pressure update on slots (i0-2 .. i0+VT)^2; its columns reach t at +0 .. +1
    for (int q = tid; q < DW * DW; q += TPB) {
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
            T acc = 0;
            static_for(std::make_integer_sequence<int, SST.n[tu]>{}, [&](auto ec) {
                constexpr int e = decltype(ec)::value;
                constexpr SEnt en = SST.e[tu][e];
                if constexpr (tfield(en.in) == 2) acc += sh.cf[SST.off[tu] + e] * sh.dp[en.in - T_PL][ty + 1 + en.dj][tx + 1 + en.di];
            });
            rv[tu] = dof_free(tu, si, sj, n) ? sh.ru[tu][ty][tx] - acc : (T)0;
        });
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NU; ++q) sh.ru[q][ty][tx] = rv[q];
    }
    __syncthreads();
    upatch_solves<T>(sh.ru, sh.ui, sh.so, i0, j0, n, tx, ty);
    __syncthreads();
    if (tx < VO && ty < VO) {
        const int si = i0 + tx, sj = j0 + ty;
        if (si <= n && sj <= n) {
            const long long s0 = slot_index(L, si, sj);
            T du[NU];
            upatch_gather<T>(sh.so, tx, ty, du);
#pragma unroll
            for (int q = 0; q < NU; ++q)
                if (dof_free(q, si, sj, n)) x[q * L.plane + s0] = (ZERO ? (T)0 : x_src[q * L.plane + s0]) + omega * du[q];
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

template <typename T, bool ZERO>
__global__ __launch_bounds__(TPB) void k_bsr_second(const T* __restrict__ r, const T* __restrict__ t,
                                                    const T* x_src, T* x, Layout L, const T* __restrict__ uinv,
                                                    const T* __restrict__ coef, const T* __restrict__ d,
                                                    T omega, T omega_J) {
    __shared__ BsrSecondLds<T> sh;
    int bx, by;
    xcd_tile(bx, by);
    bsr_second_tile<T, ZERO>(r, t, x_src, x, L, uinv, coef, d, omega, omega_J, bx, by, sh);
}

template <typename T>
void launch_bsr_step(const LevelView<T>& lv, T* x, const T* b, T* r, T* t, bool x_is_zero, bool uniform, T kinv_s,
                     T omega, T omega_J, const T* xc, const Layout* Lc, const T* pw, T* xtmp, hipStream_t st) {
    dim3 blk(TB, TB);
    dim3 grd((lv.L.n + 1 + VO - 1) / VO, (lv.L.n + 1 + VO - 1) / VO);
    const Layout lc = Lc ? *Lc : lv.L;
    if (xc && (x_is_zero || !xtmp || xtmp == x)) throw ArgError{"the prolongation needs an iterate and a buffer"};
#define BIOT_BSR_FIRST(U, Z, P)                                                                                  \
    hipLaunchKernelGGL((k_bsr_first<T, U, Z, P>), grd, blk, 0, st, x, xtmp, b, r, t, lv.L, lv.kinv, kinv_s,     \
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
    if (x_is_zero)
        hipLaunchKernelGGL((k_bsr_second<T, true>), grd, blk, 0, st, r, t, xsrc, x, lv.L, lv.uinv, lv.coef, lv.bsrd,
                           omega, omega_J);
    else
        hipLaunchKernelGGL((k_bsr_second<T, false>), grd, blk, 0, st, r, t, xsrc, x, lv.L, lv.uinv, lv.coef, lv.bsrd,
                           omega, omega_J);
}
template void launch_bsr_step<double>(const LevelView<double>&, double*, const double*, double*, double*, bool, bool,
                                      double, double, double, const double*, const Layout*, const double*, double*,
                                      hipStream_t);
template void launch_bsr_step<float>(const LevelView<float>&, float*, const float*, float*, float*, bool, bool, float,
                                     float, float, const float*, const Layout*, const float*, float*, hipStream_t);

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

template <typename T, bool UNIFORM>
__device__ __forceinline__ void residual_restrict_tile(const T* __restrict__ x, const T* __restrict__ b,
                                                       T* __restrict__ rc, const Layout& Lf, const Layout& Lc,
                                                       const T* __restrict__ kinv, T kinv_s,
                                                       const T* __restrict__ coef, const T* __restrict__ w, int bx,
                                                       int by, ResRestrictLds<T, UNIFORM>& sh) {
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TB + tx;
    const int I0 = bx * RT, J0 = by * RT;
    const int f0i = 2 * I0 - 2, f0j = 2 * J0 - 2;   // fine origin of the residual window
    const int n = Lf.n;
    {
        // x on (f0 - 1 .. f0 + RRW)^2; slots below -2 lie outside the padded plane and only
        // feed residuals of slots outside the mesh (masked)
        constexpr int NV = NTYPES * RXW * RXW;
        constexpr int NIT = (NV + TPB - 1) / TPB;
        T v[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * TPB;
            const int p = q / (RXW * RXW), rem = q - p * (RXW * RXW), bj = rem / RXW, ai = rem - bj * RXW;
            const int si = f0i - 1 + ai, sj = f0j - 1 + bj;
            v[it] = (q < NV && si >= -2 && sj >= -2 && si <= n + 1 && sj <= n + 1)
                        ? x[p * Lf.plane + slot_index(Lf, si, sj)] : (T)0;
        }
        T bv[NTYPES];
        const int si = f0i + tx, sj = f0j + ty;
        const bool inb = si >= -2 && sj >= -2 && si <= n + 1 && sj <= n + 1;
#pragma unroll
        for (int t = 0; t < NTYPES; ++t) bv[t] = inb ? b[t * Lf.plane + slot_index(Lf, si, sj)] : (T)0;
        Table<T, NSTENCIL> tcf;
        tcf.load(coef, tid);
        T kv[UNIFORM ? 1 : (2 * RXW * RXW + TPB - 1) / TPB];
        if constexpr (!UNIFORM) {
#pragma unroll
            for (int it = 0; it < (2 * RXW * RXW + TPB - 1) / TPB; ++it) {
                const int q = tid + it * TPB;
                const int p = q / (RXW * RXW), rem = q - p * (RXW * RXW), bj = rem / RXW, ai = rem - bj * RXW;
                const int ki = f0i - 1 + ai, kj = f0j - 1 + bj;
                kv[it] = (q < 2 * RXW * RXW && ki >= -2 && kj >= -2 && ki <= n + 1 && kj <= n + 1)
                             ? kinv[p * Lf.plane + slot_index(Lf, ki, kj)] : (T)0;
            }
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * TPB;
            if (q < NV) (&sh.xs[0][0][0])[q] = v[it];
        }
#pragma unroll
        for (int t = 0; t < NTYPES; ++t) sh.rs[t][ty][tx] = bv[t];
        tcf.store(sh.cf, tid);
        if constexpr (!UNIFORM) {
#pragma unroll
            for (int it = 0; it < (2 * RXW * RXW + TPB - 1) / TPB; ++it) {
                const int q = tid + it * TPB;
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
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NTYPES; ++t) sh.rs[t][ty][tx] = rv[t];
    }
    __syncthreads();
    // restriction of the tile's coarse slots: wave (q / 64) handles one coarse DoF type, so the
    // compile-time restriction row is uniform over the wave
    static_assert(RT * RT <= 64, "one coarse tile per wave");
    for (int q = tid; q < NTYPES * 64; q += TPB) {
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

template <typename T, bool UNIFORM>
__global__ __launch_bounds__(TPB) void k_residual_restrict(const T* __restrict__ x, const T* __restrict__ b,
                                                           T* __restrict__ rc, Layout Lf, Layout Lc,
                                                           const T* __restrict__ kinv, T kinv_s,
                                                           const T* __restrict__ coef, const T* __restrict__ w) {
    __shared__ ResRestrictLds<T, UNIFORM> sh;
    int bx, by;
    xcd_tile(bx, by);
    residual_restrict_tile<T, UNIFORM>(x, b, rc, Lf, Lc, kinv, kinv_s, coef, w, bx, by, sh);
}

template <typename T>
void launch_residual_restrict(const LevelView<T>& lf, const Layout& Lc, const T* x, const T* b, T* rc,
                              bool uniform, T kinv_s, const T* w, hipStream_t st, const LaunchTiming* tm) {
    dim3 blk(TB, TB);
    dim3 grd((Lc.n + 1 + RT - 1) / RT, (Lc.n + 1 + RT - 1) / RT);
    hipEvent_t e0 = tm ? tm->start : nullptr, e1 = tm ? tm->stop : nullptr;
    if (uniform)
        hipExtLaunchKernelGGL((k_residual_restrict<T, true>), grd, blk, 0, st, e0, e1, 0, x, b, rc, lf.L, Lc, lf.kinv,
                              kinv_s, lf.coef, w);
    else
        hipExtLaunchKernelGGL((k_residual_restrict<T, false>), grd, blk, 0, st, e0, e1, 0, x, b, rc, lf.L, Lc, lf.kinv,
                              kinv_s, lf.coef, w);
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

// =========================================================================================
// coarsest level: dense inverse applied by one workgroup (Sec. 5.1 direct solve)
// =========================================================================================
template <typename T>
__device__ __forceinline__ void coarse_solve_block(const double* __restrict__ AinvT, int N, const int* __restrict__ idx,
                                                   const T* __restrict__ b, T* __restrict__ x, double* bb, int tid,
                                                   int nt) {
    for (int k = tid; k < N; k += nt) bb[k] = (double)b[idx[k]];
    __syncthreads();
    for (int k = tid; k < N; k += nt) {
        double s = 0;
        for (int l = 0; l < N; ++l) s += AinvT[(long long)l * N + k] * bb[l];
        x[idx[k]] = (T)s;
    }
}

// x = A_c^{-1} b on the free DoFs of the coarsest level (AinvT: the inverse, transposed, so that
// the threads of a row step read consecutive entries)
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(const double* __restrict__ AinvT, int N,
                                                      const int* __restrict__ idx, const T* __restrict__ b,
                                                      T* __restrict__ x) {
    extern __shared__ double bb[];
    coarse_solve_block<T>(AinvT, N, idx, b, x, bb, threadIdx.x, blockDim.x);
}

template <typename T>
void launch_coarse_solve(const double* AinvT, int N, const int* idx, const T* b, T* x, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse_solve<T>, dim3(1), dim3(256), N * sizeof(double), st, AinvT, N, idx, b, x);
}

__global__ void k_transpose(const double* __restrict__ A, double* __restrict__ AT, int N) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)N * N) return;
    const int r = (int)(q / N), c = (int)(q - (long long)r * N);
    AT[(long long)c * N + r] = A[q];
}

void launch_transpose(const double* A, double* AT, int N, hipStream_t st) {
    const long long nn = (long long)N * N;
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, A, AT, N);
}

template void launch_coarse_solve<double>(const double*, int, const int*, const double*, double*, hipStream_t);
template void launch_coarse_solve<float>(const double*, int, const int*, const float*, float*, hipStream_t);

// dense coarse matrix: row k (free DoF free_idx[k] of the padded layout) from the stencil
__global__ void k_coarse_matrix(Layout L, const StencilEntry* __restrict__ st, const int* __restrict__ st_off,
                                const double* __restrict__ kinv, const int* __restrict__ free_idx,
                                const int* __restrict__ free_map, int N, double* __restrict__ A) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const long long p = free_idx[k];
    const int t = (int)(p / L.plane);
    const long long s = p - t * L.plane;
    double* row = A + (long long)k * N;
    for (int c = 0; c < N; ++c) row[c] = 0;
    for (int e = st_off[t]; e < st_off[t + 1]; ++e) {
        const StencilEntry E = st[e];
        const long long q = E.in_t * L.plane + s + (long long)E.dj * L.pitch + E.di;
        const int col = free_map[q];
        if (col < 0) continue;
        double c = E.coef;
        if (E.ktri >= 0) c *= kinv[E.ktri * L.plane + s + (long long)E.kdj * L.pitch + E.kdi];
        row[col] += c;
    }
}

void launch_coarse_matrix(const Layout& L, const StencilEntry* st_tab, const int* st_off, const double* kinv,
                          const int* free_idx, const int* free_map, int N, double* A, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse_matrix, dim3((N + 127) / 128), dim3(128), 0, st, L, st_tab, st_off, kinv,
                       free_idx, free_map, N, A);
}

// Gauss-Jordan inversion with partial pivoting, one workgroup; M is destroyed.
__global__ __launch_bounds__(256) void k_gauss_jordan(double* __restrict__ M, double* __restrict__ Inv, int N,
                                                      int* __restrict__ status) {
    extern __shared__ double fcol[];
    __shared__ double rv[256];
    __shared__ int ri[256];
    __shared__ int piv;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (long long q = tid; q < (long long)N * N; q += nt) Inv[q] = ((q / N) == (q % N)) ? 1.0 : 0.0;
    if (tid == 0) *status = 0;
    __syncthreads();
    for (int c = 0; c < N; ++c) {
        double best = -1.0;
        int bi = c;
        for (int r = c + tid; r < N; r += nt) {
            const double v = fabs(M[(long long)r * N + c]);
            if (v > best) {
                best = v;
                bi = r;
            }
        }
        rv[tid] = best;
        ri[tid] = bi;
        __syncthreads();
        if (tid == 0) {
            double b = -1.0;
            int bj = c;
            for (int q = 0; q < nt; ++q)
                if (rv[q] > b || (rv[q] == b && ri[q] < bj)) {
                    b = rv[q];
                    bj = ri[q];
                }
            piv = (b > 0.0) ? bj : -1;
            if (b <= 0.0) *status = 1;
        }
        __syncthreads();
        if (piv < 0) return;
        const int pr = piv;
        if (pr != c)
            for (int k = tid; k < N; k += nt) {
                double a = M[(long long)pr * N + k];
                M[(long long)pr * N + k] = M[(long long)c * N + k];
                M[(long long)c * N + k] = a;
                a = Inv[(long long)pr * N + k];
                Inv[(long long)pr * N + k] = Inv[(long long)c * N + k];
                Inv[(long long)c * N + k] = a;
            }
        __syncthreads();
        const double d = 1.0 / M[(long long)c * N + c];
        __syncthreads();
        for (int k = tid; k < N; k += nt) {
            M[(long long)c * N + k] *= d;
            Inv[(long long)c * N + k] *= d;
        }
        __syncthreads();
        for (int r = tid; r < N; r += nt) fcol[r] = M[(long long)r * N + c];
        __syncthreads();
        for (long long q = tid; q < (long long)N * N; q += nt) {
            const int r = (int)(q / N), k = (int)(q % N);
            if (r == c) continue;
            const double f = fcol[r];
            if (f == 0.0) continue;
            M[q] -= f * M[(long long)c * N + k];
            Inv[q] -= f * Inv[(long long)c * N + k];
        }
        __syncthreads();
    }
}

void launch_gauss_jordan(double* A, double* Inv, int N, int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(256), N * sizeof(double), st, A, Inv, N, status);
}

// =========================================================================================
// permeability: 1/K per triangle on the padded grid, and its coarsening (mean of the four
// children's 1/K, i.e. the harmonic mean of K)
// =========================================================================================
__global__ void k_kinv_from_K(const double* __restrict__ K, double Ks, double* __restrict__ kinv, Layout L) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= L.n || j >= L.n) return;
    const long long c = (long long)j * L.n + i;
    const long long nn = (long long)L.n * L.n;
    const double kl = K ? K[c] : Ks;
    const double ku = K ? K[nn + c] : Ks;
    kinv[slot_index(L, i, j)] = 1.0 / kl;
    kinv[L.plane + slot_index(L, i, j)] = 1.0 / ku;
}

void launch_kinv_from_K(const double* K_tri, double K_scalar, double* kinv, const Layout& L, hipStream_t st) {
    launch_fill(kinv, 2 * L.plane, 0.0, st);
    dim3 blk(64, 4), grd((L.n + 63) / 64, (L.n + 3) / 4);
    hipLaunchKernelGGL(k_kinv_from_K, grd, blk, 0, st, K_tri, K_scalar, kinv, L);
}

__global__ void k_kinv_coarsen(const double* __restrict__ kf, Layout Lf, double* __restrict__ kc, Layout Lc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I >= Lc.n || J >= Lc.n) return;
    const double* fL = kf;
    const double* fU = kf + Lf.plane;
    const int i = 2 * I, j = 2 * J;
    const double cl = 0.25 * (fL[slot_index(Lf, i, j)] + fL[slot_index(Lf, i + 1, j)] +
                              fL[slot_index(Lf, i, j + 1)] + fU[slot_index(Lf, i, j)]);
    const double cu = 0.25 * (fU[slot_index(Lf, i + 1, j + 1)] + fU[slot_index(Lf, i + 1, j)] +
                              fU[slot_index(Lf, i, j + 1)] + fL[slot_index(Lf, i + 1, j + 1)]);
    kc[slot_index(Lc, I, J)] = cl;
    kc[Lc.plane + slot_index(Lc, I, J)] = cu;
}

void launch_kinv_coarsen(const double* kf, const Layout& Lf, double* kc, const Layout& Lc, hipStream_t st) {
    launch_fill(kc, 2 * Lc.plane, 0.0, st);
    dim3 blk(64, 4), grd((Lc.n + 63) / 64, (Lc.n + 3) / 4);
    hipLaunchKernelGGL(k_kinv_coarsen, grd, blk, 0, st, kf, Lf, kc, Lc);
}

// =========================================================================================
// Krylov BLAS-1 (FP64, deterministic reductions)
// =========================================================================================
// ---- classical Gram-Schmidt pass: dots, update with norm, deterministic reductions ----------------
// The partial sums of each block go to partial[q * np + b] (np blocks); a second kernel adds them
// in a fixed order.  Kernels given run_if return at once when *run_if == 0.
constexpr int DOT_BLOCKS = RED_BLOCKS;     // dot-product blocks (contiguous chunks)
constexpr int UPD_BLOCKS = 4 * RED_BLOCKS; // update blocks (grid stride)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// partial sums of V_q . w (q < nv) and of w . w (slot nv), GSV vectors per pass over the chunk;
// each value is summed within a wave by a butterfly, then over the 4 waves in a fixed order
constexpr int GSV = 8;
__global__ __launch_bounds__(256) void k_gs_dots(const double* __restrict__ V, long long ldv, int nv,
                                                 const double* __restrict__ w, long long n,
                                                 double* __restrict__ partial, const double* run_if) {
    if (run_if && *run_if == 0.0) return;
    __shared__ double red[4][GSV + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    for (int v0 = 0; v0 == 0 || v0 < nv; v0 += GSV) {
        double acc[GSV + 1];
#pragma unroll
        for (int q = 0; q <= GSV; ++q) acc[q] = 0;
        for (long long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
            const double we = w[e];
#pragma unroll
            for (int q = 0; q < GSV; ++q)
                if (v0 + q < nv) acc[q] += V[(long long)(v0 + q) * ldv + e] * we;
            if (v0 == 0) acc[GSV] += we * we;
        }
#pragma unroll
        for (int q = 0; q <= GSV; ++q) {
            const double t = wave_sum(acc[q]);
            if (lane == 0) red[wave][q] = t;
        }
        __syncthreads();
        const int q = threadIdx.x;
        if (q <= GSV) {
            const double r = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
            if (q < GSV && v0 + q < nv) partial[(long long)(v0 + q) * gridDim.x + blockIdx.x] = r;
            if (q == GSV && v0 == 0) partial[(long long)nv * gridDim.x + blockIdx.x] = r;
        }
        __syncthreads();
    }
}

// w -= sum_q h[q] V_q, with partial sums of the new w . w
__global__ __launch_bounds__(256) void k_gs_update(double* __restrict__ w, const double* __restrict__ V,
                                                   long long ldv, int nv, const double* __restrict__ h,
                                                   long long n, double* __restrict__ partial,
                                                   const double* run_if) {
    if (run_if && *run_if == 0.0) return;
    __shared__ double wred[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc = 0;
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < n; e += stride) {
        double sv = w[e];
        for (int q = 0; q < nv; ++q) sv -= h[q] * V[(long long)q * ldv + e];
        w[e] = sv;
        acc += sv * sv;
    }
    const double t = wave_sum(acc);
    if (lane == 0) wred[wave] = t;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = wred[0] + wred[1] + wred[2] + wred[3];
}

// out[q] = sum_b partial[q * np + b], one block per q (fixed order); host: optional mirror.
// flag (block 0, optional): 1 when out[0] < 0.5 * prev (the Daniel-Gragg-Kaufman-Stewart test
// for a second orthogonalization pass, eta = 1/sqrt(2)).
__global__ __launch_bounds__(256) void k_gs_reduce(const double* __restrict__ partial, int np,
                                                   double* __restrict__ out, double* __restrict__ host,
                                                   const double* __restrict__ prev, double* __restrict__ flag,
                                                   const double* run_if) {
    if (run_if && *run_if == 0.0) return;
    __shared__ double wred[4];
    const int q = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double sv = 0;
    for (int b2 = threadIdx.x; b2 < np; b2 += blockDim.x) sv += partial[(long long)q * np + b2];
    const double t = wave_sum(sv);
    if (lane == 0) wred[wave] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double r = wred[0] + wred[1] + wred[2] + wred[3];
        out[q] = r;
        if (host) host[q] = r;
        if (flag) {
            *flag = (r < 0.5 * (*prev)) ? 1.0 : 0.0;
            if (host) host[1] = *flag;
        }
    }
}

void launch_gs_dots(const double* V, long long ldv, int nv, const double* w, long long n, double* partial,
                    double* out, double* host, const double* run_if, hipStream_t st) {
    hipLaunchKernelGGL(k_gs_dots, dim3(DOT_BLOCKS), dim3(256), 0, st, V, ldv, nv, w, n, partial, run_if);
    hipLaunchKernelGGL(k_gs_reduce, dim3(nv + 1), dim3(256), 0, st, partial, DOT_BLOCKS, out, host, nullptr,
                       nullptr, run_if);
}

void launch_gs_update(double* w, const double* V, long long ldv, int nv, const double* h, long long n,
                      double* partial, double* norm2, const double* prev, double* flag, double* host,
                      const double* run_if, hipStream_t st) {
    hipLaunchKernelGGL(k_gs_update, dim3(UPD_BLOCKS), dim3(256), 0, st, w, V, ldv, nv, h, n, partial, run_if);
    hipLaunchKernelGGL(k_gs_reduce, dim3(1), dim3(256), 0, st, partial, UPD_BLOCKS, norm2, host, prev, flag,
                       run_if);
}

// dst = src / sqrt(*na), or / sqrt(*nb) when sel != nullptr and *sel != 0
__global__ void k_normalize(double* __restrict__ dst, const double* __restrict__ src, long long n,
                            const double* __restrict__ na, const double* __restrict__ nb,
                            const double* __restrict__ sel) {
    const double nv = (sel && *sel != 0.0) ? *nb : *na;
    const double s = 1.0 / sqrt(nv);
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < n; e += stride) dst[e] = src[e] * s;
}

void launch_normalize(double* dst, const double* src, long long n, const double* na, const double* nb,
                      const double* sel, hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_normalize, dim3(blocks), dim3(256), 0, st, dst, src, n, na, nb, sel);
}

__global__ void k_scale(double* __restrict__ dst, const double* __restrict__ src, long long n, double s) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < n; e += stride) dst[e] = src[e] * s;
}

void launch_scale(double* dst, const double* src, long long n, double s, hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_scale, dim3(blocks), dim3(256), 0, st, dst, src, n, s);
}

__global__ void k_lincomb_add(double* __restrict__ x, const double* __restrict__ Z, long long ldz, int nv,
                              const double* __restrict__ y, long long n) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < n; e += stride) {
        double s = x[e];
        for (int q = 0; q < nv; ++q) s += y[q] * Z[(long long)q * ldz + e];
        x[e] = s;
    }
}

void launch_lincomb_add(double* x, const double* Z, long long ldz, int nv, const double* y, long long n,
                        hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_lincomb_add, dim3(blocks), dim3(256), 0, st, x, Z, ldz, nv, y, n);
}

// =========================================================================================
// adjoint gradient with respect to ln K per triangle
// =========================================================================================
__global__ void k_grad_logK(Layout L, const double* __restrict__ x, const double* __restrict__ lam,
                            const double* __restrict__ kinv, const double* __restrict__ mloc,
                            double* __restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= L.n || j >= L.n) return;
    // local RT0 DoFs of L(i,j): D(i,j), V(i,j), H(i,j); of U(i,j): H(i,j+1), D(i,j), V(i+1,j)
    const int tl[3] = {T_WD, T_WV, T_WH}, tu[3] = {T_WH, T_WD, T_WV};
    const int ul_i[3] = {0, 0, 0}, ul_j[3] = {0, 0, 0};
    const int uu_i[3] = {0, 0, 1}, uu_j[3] = {1, 0, 0};
    for (int u = 0; u < 2; ++u) {
        double wv[3], lv[3];
        for (int k = 0; k < 3; ++k) {
            const int t = u ? tu[k] : tl[k];
            const int di = u ? uu_i[k] : ul_i[k], dj = u ? uu_j[k] : ul_j[k];
            const long long o = t * L.plane + slot_index(L, i + di, j + dj);
            wv[k] = x[o];
            lv[k] = lam[o];
        }
        double s = 0;
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) s += lv[k] * mloc[u * 9 + k * 3 + l] * wv[l];
        const double ki = kinv[u * L.plane + slot_index(L, i, j)];
        g[(long long)u * L.n * L.n + (long long)j * L.n + i] = ki * s;
    }
}

void launch_grad_logK(const Layout& L, const double* x, const double* lam, const double* kinv,
                      const double* mloc, double* g_tri, hipStream_t st) {
    dim3 blk(64, 4), grd((L.n + 63) / 64, (L.n + 3) / 4);
    hipLaunchKernelGGL(k_grad_logK, grd, blk, 0, st, L, x, lam, kinv, mloc, g_tri);
}

// =========================================================================================
// layout export: the 20-slot patch table, by the index arithmetic of the Vanka kernel
// =========================================================================================
__device__ inline int canon_index(const Canon& C, int n, int t, int i, int j) {
    if (!dof_free(t, i, j, n)) return -1;
    long long r;
    if (t == T_UX || t == T_UY)
        r = (long long)(j - 1) * (n - 1) + (i - 1);
    else if (t == T_BH || t == T_WH)
        r = (long long)(j - 1) * n + i;
    else if (t == T_BV || t == T_WV)
        r = (long long)j * (n - 1) + (i - 1);
    else
        r = (long long)j * n + i;
    return (int)(C.off[t] + r);
}

__global__ void k_patch_table(Layout L, Canon C, int* __restrict__ table) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = L.n;
    const long long nv = (long long)(n + 1) * (n + 1);
    if (v >= nv) return;
    const int i = (int)(v % (n + 1)), j = (int)(v / (n + 1));
    if ((i == 0 && j == 0) || (i == n && j == n)) return;
    // row index: vertices in row-major order minus the dropped corner (0,0)
    const long long row = v - 1;
    for (int s = 0; s < PATCH; ++s) {
        int t, di, dj;
        patch_slot(s, t, di, dj);
        table[row * PATCH + s] = canon_index(C, n, t, i + di, j + dj);
    }
}

void launch_patch_table(const Layout& L, const Canon& C, int* table, hipStream_t st) {
    const long long nv = (long long)(L.n + 1) * (L.n + 1);
    hipLaunchKernelGGL(k_patch_table, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, L, C, table);
}

}  // namespace biot
