// Fused residual + additive Vanka relaxation step (Sec. 3.2.1) for gfx950: FP64 matrix-core
// products for constant permeability, per-patch elimination otherwise.
#include "tile.h"
#include "patch_solve.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace biot {

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
__device__ inline double vanka_weight(int t, int i, int j, int n) {
    if (t <= T_UY) return 1.0;
    if (t <= T_WD) return 0.5;
    if (t == T_PL) return (i == 0 && j == 0) ? 0.5 : 1.0 / 3.0;
    return (i == n - 1 && j == n - 1) ? 0.5 : 1.0 / 3.0;
}

// Whether the patch of vertex (i, j) belongs to colour code `color` of the multiplicative form.
// Two patches share a DoF only when their vertices are joined by a mesh edge, so a colouring of
// the vertex graph makes the patches of a colour disjoint.  Codes 0..3: four colours
// (i mod 2) + 2 (j mod 2); codes 4..6: three colours 4 + (i + 2 j) mod 3 (the edge neighbours
// (i +- 1, j), (i, j +- 1), (i +- 1, j -+ 1) shift i + 2 j by +-1, +-2, -+1).
__host__ __device__ constexpr bool in_color(int i, int j, int color) {
    return color < 4 ? (i & 1) + 2 * (j & 1) == color : (i + 2 * j) % 3 == color - 4;
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

// One variable-K patch solve: the patch's factors (stored, fp != nullptr, FP64 only, or formed from
// the 1/K of its star), then the solve, which reads the patch residual from the staged residual in
// LDS where it needs it (it stays there until the barrier after the patch phase).
template <typename T, typename P, bool ALLP, bool FACOK, typename KV>
__device__ __forceinline__ void vanka_patch(const DevPatchClass<P>& pc, const KV& kv, const P* __restrict__ wblk,
                                            const double* __restrict__ fp, long long plane,
                                            const T (&rs)[NTYPES][RW][RW], int tx, int ty, P (&out)[PATCH]) {
    PatchFac<P> f;
    bool stored = false;
    if constexpr (FACOK) {
        if (fp) {
            double* fv = reinterpret_cast<double*>(&f);
#pragma unroll
            for (int q = 0; q < PFAC; ++q) fv[q] = fp[(long long)q * plane];
            stored = true;
        }
    }
    if (!stored) patch_factor<P, ALLP>(pc, kv, wblk, f);
    if constexpr (sizeof(P) == 8) __asm__ volatile("" ::: "memory");
    patch_apply<P, ALLP>(
        [&](int s) {
            int t, di, dj;
            patch_slot(s, t, di, dj);
            return (P)rs[t][ty + 1 + dj][tx + 1 + di];
        },
        pc, f, out, 1);
}

// LDS of the fused step.  The staged x_in and the residual are dead once the patch residuals
// are in registers; the patch corrections then reuse their space.
template <typename T, typename P, bool UNIFORM, int NCLS, bool PROL>
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
    // patch classes of the tile (variable K)
    std::conditional_t<UNIFORM, char, DevPatchClass<P>> pcs[UNIFORM ? 1 : NCLS];
    // the coarse iterate is dead once the prolongation has been added to the staged window, before
    // the owned iterate is copied out of it
    union {
        T xcs[PROL ? NTYPES : 1][PROL ? PCW : 1][PROL ? PCW : 1];      // coarse iterate (prolongation)
        T xo[UNIFORM ? 1 : NTYPES][UNIFORM ? 1 : VO][UNIFORM ? 1 : VO];  // iterate on the owned slots (variable K)
    };
    T cf[NSTENCIL];                                              // stencil coefficients
    T pwl[PROL ? NPWEIGHTS : 1];                                 // prolongation weights
};

// PROL: the iterate is x_in + P x_c (prolongation of the coarse-grid correction, Sec. 3),
// formed on the staged window; x_out = x_in + P x_c + omega (...).
// One tile (bx, by) of the step, by the 16 x 16 x NZ threads of a block with LDS sh.  Thread
// (tx, ty, tz) stages and gathers for slot (tx, ty) the DoF types of its layer tz; the patch
// products are spread over the block's 4 NZ waves.  P: arithmetic of the variable-K patch
// eliminations (FP64, or FP32 with FP32 storage on request).
template <typename T, typename P, bool UNIFORM, bool ZERO, int NCLS, bool PROL, int NZ>
__device__ __forceinline__ void vanka_step_tile(const T* __restrict__ x_in, const T* __restrict__ b,
                                                T* __restrict__ x_out, const Layout& L, const T* __restrict__ kinv,
                                                T kinv_s, const T* __restrict__ coef,
                                                const DevPatchClass<P>* __restrict__ cls,
                                                const P* __restrict__ wblk, const double* __restrict__ minv,
                                                const double* __restrict__ fac,
                                                T omega, const T* __restrict__ xc, const Layout& Lc,
                                                const T* __restrict__ pw, int color, int bx, int by,
                                                VankaLds<T, P, UNIFORM, NCLS, PROL>& sh) {
    static_assert(!(PROL && ZERO), "the prolongation needs an iterate");
    auto& xs = sh.u.a.xs;
    auto& rs = sh.u.a.rs;
    static_assert(NZ == 1 || (NZ == 2 && UNIFORM), "two thread layers for constant K only");
    constexpr int NTH = TPB * NZ;
    const int tx = threadIdx.x, ty = threadIdx.y, tz = NZ > 1 ? (int)threadIdx.z : 0;
    const int tid = (tz * TB + ty) * TB + tx;
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
        constexpr int NIT = (NM + NTH - 1) / NTH;
        constexpr int NCL = UNIFORM ? NCLS : 1;
        const int nc = cw * (cjhi - cjlo + 1);
        double mv[NCL][NIT];
        // variable K: the tile's patch classes, as words of sizeof(P) bytes
        constexpr int NPW = sizeof(DevPatchClass<P>) / sizeof(P);
        static_assert(NPW * sizeof(P) == sizeof(DevPatchClass<P>) && NPW <= NTH, "class staging");
        constexpr int NPC = UNIFORM ? 1 : NCLS;
        P pv[NPC];
        if constexpr (!UNIFORM) {
#pragma unroll
            for (int k = 0; k < NPC; ++k) {
                const int cidx = 3 * (cjlo + k / cw) + cilo + k % cw;
                pv[k] = (k < nc && tid < NPW) ? reinterpret_cast<const P*>(cls + cidx)[tid] : (P)0;
            }
        }
        if constexpr (UNIFORM) {
#pragma unroll
            for (int k = 0; k < NCL; ++k) {
                const int cidx = 3 * (cjlo + k / cw) + cilo + k % cw;
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    const int q = tid + it * NTH;
                    mv[k][it] = (k < nc && q < NM) ? minv[cidx * NM + q] : 0.0;
                }
            }
        }
        Window<T, NTYPES, RW, NTH> wb;
        wb.load(b, L.plane, L, i0 - 1, j0 - 1, tid);
        Window<T, NTYPES, XS, NTH> wx;
        if constexpr (!ZERO) wx.load(x_in, L.plane, L, i0 - 2, j0 - 2, tid);
        Window<T, 2, KW, NTH> wk;
        if constexpr (!UNIFORM) wk.load(kinv, L.plane, L, i0 - 2, j0 - 2, tid);
        // coarse slots i0/2 - 1 .. i0/2 + PCW - 2 feed the fine window i0 - 2 .. i0 + VT + 1
        Window<T, NTYPES, PCW, NTH> wc;
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
                    const int q = tid + it * NTH;
                    if (k < nc && q < NM) sh.ms[k][q] = mv[k][it];
                }
        }
        if constexpr (!UNIFORM) {
#pragma unroll
            for (int k = 0; k < NPC; ++k)
                if (k < nc && tid < NPW) reinterpret_cast<P*>(&sh.pcs[k])[tid] = pv[k];
        }
        wb.store(&rs[0][0][0], tid);
        if constexpr (!ZERO) wx.store(&xs[0][0][0], tid);
        if constexpr (!UNIFORM) wk.store(&sh.ks[0][0][0], tid);
        if constexpr (PROL) wc.store(&sh.xcs[0][0][0], tid);
    }
    __syncthreads();
    if constexpr (PROL) {
        prolong_window<T, NTH>(xs, sh.xcs, sh.pwl, i0, j0, n, tid);
        __syncthreads();
    }
    // ---- residual r = b - A x_in of slot (i0-1+tx, j0-1+ty), zero on absent DoFs -----------------
    if constexpr (!ZERO) {
        const int si = i0 - 1 + tx, sj = j0 - 1 + ty;
        const bool in = si <= n + 1 && sj <= n + 1;
        T rv[NTYPES];
        static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
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
                acc += cc * xs[en.in][ty + 1 + en.dj][tx + 1 + en.di];
            });
            rv[t] = (in && dof_free(t, si, sj, n)) ? rs[t][ty][tx] - acc : (T)0;
        });
        static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
            if (rgroup(t, NZ) == tz) rs[t][ty][tx] = rv[t];
        });
        __syncthreads();
    }
    // ---- patch solves of the tile's vertices ----------------------------------------------------
    const int vi = i0 + tx, vj = j0 + ty;
    const bool patch = tx < VT && ty < VT;
    // the iterate on the owned slots, for the gather: in registers for constant K; in LDS for
    // variable K, whose patch solves need the registers (the staged window is overwritten by the
    // patch corrections)
    T xown[UNIFORM ? NTYPES : 1];
    if constexpr (UNIFORM) {
#pragma unroll
        for (int t = 0; t < NTYPES; ++t)
            xown[t] = (ZERO || !patch || ggroup(t, NZ) != tz) ? (T)0 : xs[t][ty + 2][tx + 2];
    } else if (!ZERO && tx < VO && ty < VO) {
#pragma unroll
        for (int t = 0; t < NTYPES; ++t) sh.xo[t][ty][tx] = xs[t][ty + 2][tx + 2];
    }
    // Constant K: FP64 class inverses on the matrix cores for either storage precision T.
    if constexpr (UNIFORM) {
        // The products run over batches of up to 16 patches that share one class inverse: each
        // tile row (its patches at interior-class columns), each boundary column of the tile
        // (its patches at interior-class rows) and each corner patch.  Of the NW waves, wave w
        // takes rows w, w + NW, ... and the boundary batches dealt to it (the i-th present one
        // goes to wave NW - 1 - i % NW), so a boundary tile costs one product per batch, not one
        // per class present in a row.
        constexpr int NW = 4 * NZ;                 // waves of the block
        constexpr int RPW = (VT + NW - 1) / NW;    // row batches per wave
        constexpr int EPW = (6 + NW - 1) / NW;     // boundary batches per wave
        constexpr int NB = RPW + EPW;
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
        // batch slots of this wave: 0..RPW-1 rows, then EPW boundary batches (e index, or -1)
        int ex0 = -1, ex1 = -1;
        {
            int cnt = 0;
#pragma unroll
            for (int e = 0; e < 6; ++e)
                if (epr(e)) {
                    if (cnt == NW - 1 - wave) ex0 = e;
                    if (EPW > 1 && cnt == 2 * NW - 1 - wave) ex1 = e;
                    ++cnt;
                }
        }
        // batch s: active, class (cj, ci), the lane's patch (pti, ptj) and whether it belongs to it
        auto batch = [&](int s, bool& act, int& cj, int& ci, int& pti, int& ptj, bool& own) {
            if (s < RPW) {
                ptj = wave + NW * s;
                pti = jl;
                act = ptj < VT && j0 + ptj <= n;
                cj = act ? vcls(j0 + ptj) : 1;
                ci = 1;
                own = act && pti < VT && i0 + pti <= n && vcls(i0 + pti) == 1;
            } else {
                const int e = s == RPW ? ex0 : ex1;
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
        double bf[NB][5];
#pragma unroll
        for (int sb = 0; sb < NB; ++sb) {
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
        for (int sb = 0; sb < NB; ++sb) {
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
            // rows a = kq + 4 v + 16 mb of the lane's patch; a colour step keeps its colour's
            // patches only
            if (own) {
                const bool keep = color < 0 || in_color(i0 + pti, j0 + ptj, color);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    sh.u.so[kq + 4 * v][ptj][pti] = keep ? (T)acc0[v] : (T)0;
                    if (kq + 4 * v + 16 < PATCH) sh.u.so[kq + 4 * v + 16][ptj][pti] = keep ? (T)acc1[v] : (T)0;
                }
            }
        }
    } else {
        // per-patch elimination (permeability varies from patch to patch) in precision P, class
        // data from LDS.  A tile that meets no boundary holds interior-class patches only, every
        // slot present.  With fac (FP64, the small levels): the permeability-dependent factors of
        // the patch were formed at set-up (k_patch_factors) and are only applied here, which
        // shortens the dependent chain that bounds a launch on a few tiles; otherwise they are
        // formed on the spot.
        constexpr bool FACOK = std::is_same_v<P, double>;
        P out[PATCH];
#pragma unroll
        for (int s = 0; s < PATCH; ++s) out[s] = 0;
        const bool inner = cilo == 1 && cihi == 1 && cjlo == 1 && cjhi == 1;
        const bool act = patch && vi <= n && vj <= n && (color < 0 || in_color(vi, vj, color));
        if (act) {
            // 1/K of the star triangles, read from the staged field where the factorization uses it
            auto kv = [&](int kq) {
                int ut, di, dj;
                star_tri(kq, ut, di, dj);
                return (P)sh.ks[ut][ty + 2 + dj][tx + 2 + di];
            };
            const double* fp = (FACOK && fac) ? fac + slot_index(L, vi, vj) : nullptr;
            if (inner) {
                vanka_patch<T, P, true, FACOK>(sh.pcs[0], kv, wblk, fp, L.plane, rs, tx, ty, out);
            } else {
                const int ci = vi == 0 ? 0 : (vi == n ? 2 : 1);
                const int cj = vj == 0 ? 0 : (vj == n ? 2 : 1);
                const DevPatchClass<P>& pc = sh.pcs[(cj - cjlo) * cw + (ci - cilo)];
                bool keep = false;
#pragma unroll
                for (int s = 0; s < 14; ++s) keep = keep || pc.present[s];
                if (keep) vanka_patch<T, P, false, FACOK>(pc, kv, wblk, fp, L.plane, rs, tx, ty, out);
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
            if (ggroup(T_BD, NZ) == tz) {          // layer of the displacement types
                c[T_UX] = so[0][ty][tx];
                c[T_UY] = so[1][ty][tx];
                c[T_BH] = so[3][ty][tx] + so[2][ty][tx + 1];
                c[T_BV] = so[5][ty][tx] + so[4][ty + 1][tx];
                c[T_BD] = so[6][ty][tx + 1] + so[7][ty + 1][tx];
            }
            if (ggroup(T_PU, NZ) == tz) {          // layer of the Darcy and pressure types
                c[T_WH] = so[9][ty][tx] + so[8][ty][tx + 1];
                c[T_WV] = so[11][ty][tx] + so[10][ty + 1][tx];
                c[T_WD] = so[12][ty][tx + 1] + so[13][ty + 1][tx];
                c[T_PL] = so[14][ty][tx] + so[15][ty][tx + 1] + so[16][ty + 1][tx];
                c[T_PU] = so[17][ty + 1][tx + 1] + so[18][ty][tx + 1] + so[19][ty + 1][tx];
            }
            const long long s0 = slot_index(L, si, sj);
            static_for(std::make_integer_sequence<int, NTYPES>{}, [&](auto tc) {
                constexpr int t = decltype(tc)::value;
                if (ggroup(t, NZ) == tz && dof_free(t, si, sj, n))
                    x_out[t * L.plane + s0] =
                        (ZERO ? (T)0 : (UNIFORM ? xown[UNIFORM ? t : 0] : sh.xo[UNIFORM ? 0 : t][UNIFORM ? 0 : ty][UNIFORM ? 0 : tx])) +
                        omega * (color < 0 ? (T)vanka_weight(t, si, sj, n) : (T)1) * c[t];
            });
        }
    }
}

// Two waves per SIMD for the per-patch eliminations (two tiles per CU, one tile's latency-bound
// phases overlapping the other's): in FP64 the compiler then keeps about 50 of the elimination's
// values in scratch, which costs less than the second tile gains (768 us against 1092 us per
// colour step at 2048^2 with one wave per SIMD).
template <typename T, typename P, bool UNIFORM, bool ZERO, int NCLS, bool PROL, int NZ>
__global__ __launch_bounds__(TPB * NZ, NZ == 2 ? 4 : 2) void k_vanka_step(const T* __restrict__ x_in, const T* __restrict__ b,
                                                    T* __restrict__ x_out, Layout L, const T* __restrict__ kinv,
                                                    T kinv_s, const T* __restrict__ coef,
                                                    const DevPatchClass<P>* __restrict__ cls,
                                                    const P* __restrict__ wblk,
                                                    const double* __restrict__ minv,
                                                    const double* __restrict__ fac, T omega,
                                                    const T* __restrict__ xc, Layout Lc,
                                                    const T* __restrict__ pw, int color) {
    __shared__ VankaLds<T, P, UNIFORM, NCLS, PROL> sh;
    int bx, by;
    xcd_tile(bx, by);
    vanka_step_tile<T, P, UNIFORM, ZERO, NCLS, PROL, NZ>(x_in, b, x_out, L, kinv, kinv_s, coef, cls, wblk, minv, fac,
                                                      omega, xc, Lc, pw, color, bx, by, sh);
}

// thread layers of the constant-K step (two: 512 threads per tile, each phase split over twice
// the waves; variable K keeps one layer, its per-patch eliminations already fill a layer at two
// waves per SIMD)
constexpr int VANKA_LAYERS = 2;

template <typename T, typename P, bool UNIFORM, bool ZERO, bool PROL>
static void launch_vanka_step_t(const LevelView<T>& lv, const T* x_in, const T* b, T* x_out, T kinv_s, T omega,
                                const T* xc, const Layout& Lc, const T* pw, const LaunchTiming* tm, hipStream_t st,
                                int color) {
    constexpr int NZ = UNIFORM ? VANKA_LAYERS : 1;
    dim3 blk(TB, TB, NZ);
    dim3 grd((lv.L.n + 1 + VO - 1) / VO, (lv.L.n + 1 + VO - 1) / VO);
    hipEvent_t e0 = tm ? tm->start : nullptr, e1 = tm ? tm->stop : nullptr;
    const DevPatchClass<P>* cls;
    const P* wblk;
    if constexpr (std::is_same_v<P, float>) {
        cls = lv.cls32;
        wblk = lv.wblk32;
    } else {
        cls = lv.cls;
        wblk = lv.wblk;
    }
    // a tile spans at most two vertex classes per direction unless it covers the whole mesh
    if (lv.L.n + 1 <= VT)
        hipExtLaunchKernelGGL((k_vanka_step<T, P, UNIFORM, ZERO, 9, PROL, NZ>), grd, blk, 0, st, e0, e1, 0, x_in, b,
                              x_out, lv.L, lv.kinv, kinv_s, lv.coef, cls, wblk, lv.minv, lv.fac, omega, xc, Lc,
                              pw, color);
    else
        hipExtLaunchKernelGGL((k_vanka_step<T, P, UNIFORM, ZERO, 4, PROL, NZ>), grd, blk, 0, st, e0, e1, 0, x_in, b,
                              x_out, lv.L, lv.kinv, kinv_s, lv.coef, cls, wblk, lv.minv, lv.fac, omega, xc, Lc,
                              pw, color);
}

// the ZERO / PROL forms of one (T, P, UNIFORM)
template <typename T, typename P, bool UNIFORM>
static void launch_vanka_forms(const LevelView<T>& lv, const T* x_in, const T* b, T* x_out, T kinv_s, T omega,
                               const T* xc, const Layout& lc, const T* pw, const LaunchTiming* tm, hipStream_t st,
                               int color) {
    if (xc)
        launch_vanka_step_t<T, P, UNIFORM, false, true>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st, color);
    else if (x_in)
        launch_vanka_step_t<T, P, UNIFORM, false, false>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st, color);
    else
        launch_vanka_step_t<T, P, UNIFORM, true, false>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st, color);
}

template <typename T>
void launch_vanka_step(const LevelView<T>& lv, const T* x_in, const T* b, T* x_out, bool uniform, T kinv_s,
                       T omega, hipStream_t st, const T* xc, const Layout* Lc, const T* pw, const LaunchTiming* tm,
                       int color) {
    if (color < -1 || color > 6) throw ArgError{"Vanka colour code: -1 (additive), 0..3 or 4..6"};
    const Layout lc = Lc ? *Lc : lv.L;
    if (xc && !x_in) throw ArgError{"the prolongation needs an iterate"};
    if (uniform) {
        launch_vanka_forms<T, double, true>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st, color);
        return;
    }
    if constexpr (std::is_same_v<T, float>) {
        if (lv.patch32) {
            launch_vanka_forms<T, float, false>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st, color);
            return;
        }
    }
    launch_vanka_forms<T, double, false>(lv, x_in, b, x_out, kinv_s, omega, xc, lc, pw, tm, st, color);
}

// ---- permeability-dependent patch factors (set-up and re-assembly) ---------------------------------
// One thread per vertex (i, j) of [0, n]^2: the factors of its patch (patch_factor) from the
// vertex class and the 1/K of its six star triangles; vertices without a patch are skipped.
__global__ __launch_bounds__(256) void k_patch_factors(Layout L, const double* __restrict__ kinv,
                                                       const DevPatchClass<double>* __restrict__ cls,
                                                       const double* __restrict__ wblk, double* __restrict__ fac) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int n = L.n;
    if (i > n || j > n) return;
    const int ci = i == 0 ? 0 : (i == n ? 2 : 1);
    const int cj = j == 0 ? 0 : (j == n ? 2 : 1);
    const DevPatchClass<double>& pc = cls[3 * cj + ci];
    bool keep = false;
#pragma unroll
    for (int s = 0; s < 14; ++s) keep = keep || pc.present[s];
    if (!keep) return;
    double kv[6];
#pragma unroll
    for (int kq = 0; kq < 6; ++kq) {
        int ut, di, dj;
        star_tri(kq, ut, di, dj);
        kv[kq] = kinv[ut * L.plane + slot_index(L, i + di, j + dj)];
    }
    PatchFac<double> f;
    if (ci == 1 && cj == 1)
        patch_factor<double, true>(pc, kv, wblk, f);
    else
        patch_factor<double>(pc, kv, wblk, f);
    const double* fv = reinterpret_cast<const double*>(&f);
    double* fp = fac + slot_index(L, i, j);
#pragma unroll
    for (int q = 0; q < PFAC; ++q) fp[(long long)q * L.plane] = fv[q];
}

void launch_patch_factors(const LevelView<double>& lv, double* fac, hipStream_t st) {
    dim3 blk(64, 4), grd((lv.L.n + 1 + 63) / 64, (lv.L.n + 1 + 3) / 4);
    hipLaunchKernelGGL(k_patch_factors, grd, blk, 0, st, lv.L, lv.kinv, lv.cls, lv.wblk, fac);
}
template void launch_vanka_step<double>(const LevelView<double>&, const double*, const double*, double*, bool,
                                        double, double, hipStream_t, const double*, const Layout*, const double*,
                                        const LaunchTiming*, int);
template void launch_vanka_step<float>(const LevelView<float>&, const float*, const float*, float*, bool, float,
                                       float, hipStream_t, const float*, const Layout*, const float*,
                                       const LaunchTiming*, int);

}  // namespace biot
