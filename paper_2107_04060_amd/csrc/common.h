// Shared definitions of the MI355X RQ-Biot multigrid library: DoF types, the padded
// structure-of-arrays layout, host-side table types and error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

namespace biot {

// ---- DoF types anchored at a slot (i, j) ------------------------------------------------
// Slot (i, j) anchors vertex (i, j), edges H(i, j), V(i, j), D(i, j) and triangles
// L(i, j), U(i, j).  Ten planes, one per type.
enum DofType : int {
    T_UX = 0, T_UY = 1, T_BH = 2, T_BV = 3, T_BD = 4,
    T_WH = 5, T_WV = 6, T_WD = 7, T_PL = 8, T_PU = 9
};
constexpr int NTYPES = 10;

// ---- padded layout ------------------------------------------------------------------------
// Each plane holds (n + 4) rows of `pitch` entries; slot (i, j), -2 <= i, j <= n + 1,
// lives at (j + 2) * pitch + (i + 2) (two ghost rows/columns below, one above, so that
// every gather of a transfer or stencil stays inside the plane without bounds checks).
// Entries of absent or Dirichlet DoFs and of the ghost ring are zero in every vector at
// all times.
struct Layout {
    int n;          // cells per side
    int pitch;      // entries per row (>= n + 4, multiple of 16)
    int rows;       // n + 4
    long long plane;// pitch * rows
    long long len;  // 10 * plane
};

inline Layout make_layout(int n) {
    Layout L;
    L.n = n;
    L.rows = n + 4;
    L.pitch = ((n + 4 + 15) / 16) * 16;
    L.plane = (long long)L.pitch * L.rows;
    L.len = NTYPES * L.plane;
    return L;
}

__host__ __device__ inline long long slot_index(const Layout& L, int i, int j) {
    return (long long)(j + 2) * L.pitch + (i + 2);
}

// Is the DoF of type t anchored at slot (i, j) free (exists and is not Dirichlet)?
__host__ __device__ inline bool dof_free(int t, int i, int j, int n) {
    switch (t) {
        case T_UX: case T_UY:
            return i >= 1 && i <= n - 1 && j >= 1 && j <= n - 1;
        case T_BH: case T_WH:
            return i >= 0 && i <= n - 1 && j >= 1 && j <= n - 1;
        case T_BV: case T_WV:
            return i >= 1 && i <= n - 1 && j >= 0 && j <= n - 1;
        default:  // D edges, L and U triangles
            return i >= 0 && i <= n - 1 && j >= 0 && j <= n - 1;
    }
}

// Canonical block sizes and offsets (canonical free-DoF order of the ABI).
struct Canon {
    long long size[NTYPES];
    long long off[NTYPES + 1];
};

inline Canon make_canon(int n) {
    Canon c;
    long long nv = (long long)(n - 1) * (n - 1), ne = (long long)n * (n - 1), nd = (long long)n * n;
    long long s[NTYPES] = {nv, nv, ne, ne, nd, ne, ne, nd, nd, nd};
    c.off[0] = 0;
    for (int t = 0; t < NTYPES; ++t) {
        c.size[t] = s[t];
        c.off[t + 1] = c.off[t] + s[t];
    }
    return c;
}

// ---- operator stencil ---------------------------------------------------------------------
// y[out](i, j) = sum_e coef_e * (ktri_e >= 0 ? Kinv[ktri_e](i + kdi_e, j + kdj_e) : 1)
//                          * x[in_e](i + di_e, j + dj_e)
struct StencilEntry {
    int8_t out_t, in_t, di, dj;
    int8_t ktri, kdi, kdj, pad;   // ktri: -1 none, 0 = 1/K of L, 1 = 1/K of U
    double coef;
};

// ---- transfer gather tables -----------------------------------------------------------------
// Prolongation: fine DoF (t_f) at fine slot (2I + pi, 2J + pj) receives
//   w * x_c[t_c](I + dI, J + dJ).
struct ProlongEntry {
    int8_t t_f, pi, pj, t_c, dI, dJ, pad0, pad1;
    double w;
};
// Restriction: coarse DoF t_c at coarse slot (I, J) receives w * r_f[t_f](2I + di, 2J + dj).
struct RestrictEntry {
    int8_t t_c, t_f, di, dj, pad0, pad1, pad2, pad3;
    double w;
};

// ---- Vanka patch ------------------------------------------------------------------------------
// Slot order of the 20-DoF vertex patch of vertex (i, j): type and slot offset.
constexpr int PATCH = 20;
__host__ __device__ inline void patch_slot(int s, int& t, int& di, int& dj) {
    const int tt[PATCH] = {T_UX, T_UY, T_BH, T_BH, T_BV, T_BV, T_BD, T_BD,
                           T_WH, T_WH, T_WV, T_WV, T_WD, T_WD,
                           T_PL, T_PL, T_PL, T_PU, T_PU, T_PU};
    const int ddi[PATCH] = {0, 0, -1, 0, 0, 0, -1, 0, -1, 0, 0, 0, -1, 0, 0, -1, 0, -1, -1, 0};
    const int ddj[PATCH] = {0, 0, 0, 0, -1, 0, 0, -1, 0, 0, -1, 0, 0, -1, 0, 0, -1, -1, 0, -1};
    t = tt[s];
    di = ddi[s];
    dj = ddj[s];
}

// Per-class constant patch data (class = position of the vertex: 0 low edge, 1 interior,
// 2 high edge, in each direction).  Entries of absent DoFs are identity / zero.
struct PatchClass {
    double Ainv[8][8];   // inverse of the displacement block (identity on absent DoFs)
    double H[8][6];      // Ainv * Bh^T, Bh = patch block (p rows, u cols) of A
    double G[6][6];      // Bh * Ainv * Bh^T
    double Q[6][6];      // patch block (p rows, w cols) of A  (= tau B_w)
    double c[6];         // -(patch block (p, p) of A) diagonal = (1/M) |T|
    int present[PATCH];  // 1 if the slot's DoF is free
    double weight[PATCH];// natural weight 1 / (number of patches holding the DoF)
};

// The two star edges (patch w-slot index 0..5) of each star triangle k (slot order 14..19),
// star_wpair(k, 0) and star_wpair(k, 1):
// L(i,j): H(i,j), V(i,j); L(i-1,j): H(i-1,j), D(i-1,j); L(i,j-1): V(i,j-1), D(i,j-1);
// U(i-1,j-1): V(i,j-1), H(i-1,j); U(i-1,j): V(i,j), D(i-1,j); U(i,j-1): H(i,j), D(i,j-1).
__host__ __device__ constexpr int star_wpair(int k, int p) {
    return p == 0 ? (k == 0 ? 1 : k == 1 ? 0 : k == 2 ? 2 : k == 3 ? 2 : k == 4 ? 3 : 1)
                  : (k == 0 ? 3 : k == 1 ? 4 : k == 2 ? 5 : k == 3 ? 0 : k == 4 ? 4 : 5);
}

// Runtime w-w block of a patch: W[a][b] += coef * Kinv(star triangle k).
struct WEntry {
    int8_t a, b, k, pad;
    int pad2;
    double coef;
};

// Star triangles of vertex (i, j) in patch slot order 14..19: type (0 L, 1 U) and offset.
__host__ __device__ inline void star_tri(int k, int& ut, int& di, int& dj) {
    const int uu[6] = {0, 0, 0, 1, 1, 1};
    const int ddi[6] = {0, -1, 0, -1, -1, 0};
    const int ddj[6] = {0, 0, -1, -1, 0, -1};
    ut = uu[k];
    di = ddi[k];
    dj = ddj[k];
}

// Displacement-only (8-DoF) patch data for the BSR smoother.
struct UPatchClass {
    double Ainv[8][8];
    int present[8];
    double weight[8];
};

// ---- error plumbing -------------------------------------------------------------------------------
void set_error(const std::string& msg);

struct HipError {
    hipError_t e;
    const char* what;
};

#define BIOT_HIP(call)                                                        \
    do {                                                                      \
        hipError_t _e = (call);                                               \
        if (_e != hipSuccess) throw ::biot::HipError{_e, #call};              \
    } while (0)

struct ArgError {
    std::string msg;
};
struct SingularError {
    std::string msg;
};

// ---- host-side table construction (host_tables.cpp) ------------------------------------------
struct PhysParams {
    double lambda, mu, alpha, inv_M, mu_f, tau;
};

// Stencil of the rediscretized operator on a mesh with cell size h: coefficients in the
// order of the compile-time structure (structure.h), and as an explicit entry list.
std::vector<StencilEntry> build_stencil(const PhysParams& p, double h);
// Stencil coefficients in the order of the compile-time structure (structure.h).
void build_stencil_coef(const PhysParams& p, double h, double* coef);
// Prolongation weights per (fine type, parity, coarse local DoF), see structure.h.
void build_prolong_weights(double* w);
// Gather tables of P (fine n -> coarse n/2); independent of h and of the parameters.
void build_transfer_tables(std::vector<ProlongEntry>& pro, std::vector<RestrictEntry>& res);
// Vanka class data (9 classes, index 3 * cj + ci) and w-block entries for mesh size n.
void build_patch_classes(const std::vector<StencilEntry>& st, int n, PatchClass cls[9],
                         std::vector<WEntry>& wentries);
void build_upatch_classes(const std::vector<StencilEntry>& st, int n, UPatchClass cls[9]);

}  // namespace biot
