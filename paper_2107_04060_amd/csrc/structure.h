// Compile-time structure of the rediscretized operator stencil and of the block
// prolongation, derived from the local DoF maps of the two triangles of a square.  Only the
// coefficients are computed at run time (host_tables.cpp); the kernels unroll over these
// tables, so every load offset and every coupling is a constant.
#pragma once
#include "common.h"

#include <utility>

namespace biot {

// Local DoF k of triangle u (0 = L, 1 = U) of square (0, 0): type and anchoring slot.
// Order: [ux(v0..2), uy(v0..2), bubble(e0..2), rt0(e0..2), p], edge k opposite vertex k.
// L = {(0,0), (1,0), (0,1)}: e0 = D(0,0), e1 = V(0,0), e2 = H(0,0).
// U = {(1,0), (1,1), (0,1)}: e0 = H(0,1), e1 = D(0,0), e2 = V(1,0).
struct LDof {
    int t, di, dj;
};

__host__ __device__ constexpr LDof ldof(int u, int k) {
    // vertices
    const int vl[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    const int vu[3][2] = {{1, 0}, {1, 1}, {0, 1}};
    // edges: (kind 0 H / 1 V / 2 D, slot)
    const int el[3][3] = {{2, 0, 0}, {1, 0, 0}, {0, 0, 0}};
    const int eu[3][3] = {{0, 0, 1}, {2, 0, 0}, {1, 1, 0}};
    if (k < 6) {
        const int a = k % 3;
        const int t = k < 3 ? T_UX : T_UY;
        return u == 0 ? LDof{t, vl[a][0], vl[a][1]} : LDof{t, vu[a][0], vu[a][1]};
    }
    if (k < 12) {
        const int e = (k - 6) % 3;
        const int kind = u == 0 ? el[e][0] : eu[e][0];
        const int di = u == 0 ? el[e][1] : eu[e][1];
        const int dj = u == 0 ? el[e][2] : eu[e][2];
        const int t = (k < 9 ? T_BH : T_WH) + kind;
        return LDof{t, di, dj};
    }
    return LDof{u == 0 ? T_PL : T_PU, 0, 0};
}

__host__ __device__ constexpr int lfield(int k) { return k < 9 ? 0 : (k < 12 ? 1 : 2); }
__host__ __device__ constexpr int tfield(int t) { return t <= T_BD ? 0 : (t <= T_WD ? 1 : 2); }
// pairs of local DoFs coupled by the element matrix (displacement and Darcy velocity do
// not couple; everything else may)
__host__ __device__ constexpr bool lcoupled(int a, int b) {
    return !((lfield(a) == 0 && lfield(b) == 1) || (lfield(a) == 1 && lfield(b) == 0));
}
// couplings scaled by 1/K of the triangle (RT0 mass)
__host__ __device__ constexpr bool lkdep(int a, int b) { return lfield(a) == 1 && lfield(b) == 1; }

// ---- operator stencil ---------------------------------------------------------------------
constexpr int MAXS = 48;

struct SEnt {
    int in, di, dj, kt, kdi, kdj;
};

struct StencilStruct {
    int n[NTYPES];
    int off[NTYPES + 1];
    SEnt e[NTYPES][MAXS];
};

__host__ __device__ constexpr bool sent_eq(const SEnt& a, const SEnt& b) {
    return a.in == b.in && a.di == b.di && a.dj == b.dj && a.kt == b.kt && a.kdi == b.kdi && a.kdj == b.kdj;
}

// Entry index of a coupling (row type t, local row k of triangle u in square (si, sj),
// local column k2) in the stencil, or -1.
__host__ __device__ constexpr SEnt stencil_key(int u, int si, int sj, int k2, bool kd) {
    const LDof c = ldof(u, k2);
    return kd ? SEnt{c.t, si + c.di, sj + c.dj, u, si, sj} : SEnt{c.t, si + c.di, sj + c.dj, -1, 0, 0};
}

__host__ __device__ constexpr StencilStruct make_stencil_struct() {
    StencilStruct S{};
    for (int t = 0; t < NTYPES; ++t) {
        S.n[t] = 0;
        for (int sj = -1; sj <= 0; ++sj)
            for (int si = -1; si <= 0; ++si)
                for (int u = 0; u < 2; ++u)
                    for (int k = 0; k < 13; ++k) {
                        const LDof r = ldof(u, k);
                        if (r.t != t || si + r.di != 0 || sj + r.dj != 0) continue;
                        for (int k2 = 0; k2 < 13; ++k2) {
                            if (!lcoupled(k, k2)) continue;
                            const SEnt en = stencil_key(u, si, sj, k2, lkdep(k, k2));
                            bool found = false;
                            for (int q = 0; q < S.n[t]; ++q)
                                if (sent_eq(S.e[t][q], en)) found = true;
                            if (!found) S.e[t][S.n[t]++] = en;
                        }
                    }
    }
    S.off[0] = 0;
    for (int t = 0; t < NTYPES; ++t) S.off[t + 1] = S.off[t] + S.n[t];
    return S;
}

constexpr StencilStruct SST = make_stencil_struct();
constexpr int NSTENCIL = SST.off[NTYPES];

__host__ __device__ constexpr int max_row() {
    int m = 0;
    for (int t = 0; t < NTYPES; ++t) m = SST.n[t] > m ? SST.n[t] : m;
    return m;
}
static_assert(max_row() < MAXS, "stencil row capacity");

template <typename T>
struct StencilCoef {
    T c[NSTENCIL];
};

// ---- prolongation ----------------------------------------------------------------------------
// The fine DoF of type t anchored at fine slot (2I + pi, 2J + pj) lies in the closed coarse
// square (I, J); it takes its interpolated value from one designated coarse triangle of that
// square (any coarse triangle containing it gives the same value): the one containing the
// DoF's location shifted by (+e, +2e).  Positions in units of fine h / 6.
__host__ __device__ constexpr int fine_tri(int t, int pi, int pj) {
    const int ox[NTYPES] = {0, 0, 3, 0, 3, 3, 0, 3, 2, 4};
    const int oy[NTYPES] = {0, 0, 0, 3, 3, 0, 3, 3, 2, 4};
    const int s = 6 * pi + ox[t] + 6 * pj + oy[t];
    return s < 12 ? 0 : 1;  // on the diagonal (s == 12) the shift moves the point into U
}

// number of coarse local DoFs of the field of type t, and the first local index
__host__ __device__ constexpr int fcount(int t) { return tfield(t) == 0 ? 9 : (tfield(t) == 1 ? 3 : 1); }
__host__ __device__ constexpr int ffirst(int t) { return tfield(t) == 0 ? 0 : (tfield(t) == 1 ? 9 : 12); }
// weight slot of (fine type, parity, field-local coarse DoF q)
__host__ __device__ constexpr int woff(int t) {
    return t <= T_BD ? t * 36 : (t <= T_WD ? 180 + (t - T_WH) * 12 : 216 + (t - T_PL) * 4);
}
__host__ __device__ constexpr int widx(int t, int pi, int pj, int q) {
    return woff(t) + (pj * 2 + pi) * fcount(t) + q;
}
constexpr int NPWEIGHTS = 224;

template <typename T>
struct ProlongWeights {
    T w[NPWEIGHTS];
};

// Restriction (transpose of the prolongation) in gather form: the coarse DoF of type tc at
// coarse slot (I, J) receives w[widx] * r_f[tf](2I + di, 2J + dj) for every term.
struct RTerm {
    int tf, di, dj, w;
};
constexpr int MAXR = 64;
struct RestrictStruct {
    int n[NTYPES];
    RTerm e[NTYPES][MAXR];
};

__host__ __device__ constexpr RestrictStruct make_restrict_struct() {
    RestrictStruct R{};
    for (int tc = 0; tc < NTYPES; ++tc) {
        R.n[tc] = 0;
        for (int tf = 0; tf < NTYPES; ++tf) {
            if (tfield(tf) != tfield(tc)) continue;
            for (int pj = 0; pj < 2; ++pj)
                for (int pi = 0; pi < 2; ++pi) {
                    const int u = fine_tri(tf, pi, pj);
                    for (int q = 0; q < fcount(tf); ++q) {
                        const LDof c = ldof(u, ffirst(tf) + q);
                        if (c.t != tc) continue;
                        R.e[tc][R.n[tc]++] = RTerm{tf, pi - 2 * c.di, pj - 2 * c.dj, widx(tf, pi, pj, q)};
                    }
                }
        }
    }
    return R;
}

constexpr RestrictStruct RST = make_restrict_struct();

__host__ __device__ constexpr int max_rrow() {
    int m = 0;
    for (int t = 0; t < NTYPES; ++t) m = RST.n[t] > m ? RST.n[t] : m;
    return m;
}
static_assert(max_rrow() <= MAXR, "restriction row capacity");

}  // namespace biot
