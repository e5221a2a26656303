// General-boundary path: compressed-row (CSR) operators, CSR grid transfers and explicit
// vertex-patch inverses, for boundary conditions under which the translation-invariant
// stencil of the structured path does not hold (natural conditions on part of the boundary:
// Terzaghi's column of Sec. 5, loaded and drained on one face).
//
// Paper: Sec. 2.1 (spaces, block_form), Sec. 2.3 (block_form_rq), Sec. 3 (eq. block_interp,
// R = P^T, rediscretized coarse operators), Sec. 3.1 (divergence-preserving P_u), Sec. 3.2.1
// (additive Vanka on 20-DoF vertex patches), Sec. 5 (Terzaghi's problem: its boundary
// conditions, M = infinity and the shifted Vanka blocks).
#pragma once
#include "common.h"

#include <vector>

namespace biot {

constexpr int BC_DIRICHLET = 0;   // u = 0 and w.n = 0 on the whole boundary (Sec. 5.1)
constexpr int BC_TERZAGHI = 1;    // x = 0 loaded and drained (u, w.n free), x = 1 fixed and
                                  // impermeable, y = 0 and y = 1 rollers (u_y = 0), impermeable

// Free-DoF numbering of the n x n mesh under boundary conditions bc: the full numbering in
// the canonical block order [ux, uy (vertices), bH, bV, bD, wH, wV, wD (edges), pL, pU], each
// block row-major in (j, i), with the eliminated DoFs skipped.
struct FreeMap {
    int n = 0, bc = 0;
    long long full_off[NTYPES + 1] = {};
    std::vector<int> free_of_full;   // -1: eliminated
    int N = 0;                       // free DoFs
    long long block[NTYPES] = {};    // free DoFs per type
    int n_u = 0, n_w = 0, n_p = 0;
    // free index of the DoF of type t anchored at slot (i, j), -1 if it does not exist or is
    // eliminated
    int index(int t, int i, int j) const;
};
FreeMap make_free_map(int n, int bc);

struct CsrHost {
    int rows = 0, cols = 0;
    std::vector<int> ptr, col;
    std::vector<double> val;
};

// Rediscretized operator on one level: the CSR pattern (columns sorted in each row), its
// permeability-independent values, and per entry the list of (triangle, coefficient) whose
// sum times 1/K of the triangle is the permeability-dependent part (tau mu_f M_w).
// Triangle index: L(i, j) = j n + i, U(i, j) = n^2 + j n + i.
struct OperatorHost {
    CsrHost A;
    std::vector<int> kptr, ktri;
    std::vector<double> kcoef;
};
OperatorHost build_operator(const FreeMap& m, const PhysParams& p);

// P (fine free x coarse free), the block prolongation restricted to the free DoFs of both
CsrHost build_prolongation(const FreeMap& fine, const FreeMap& coarse);
CsrHost csr_transpose(const CsrHost& a);

// 20-slot vertex patches (slot order of the layout export in the ABI), -1 for absent or
// eliminated DoFs; only vertices whose patch holds a free displacement or Darcy DoF are kept,
// in row-major (j, i) order.  Returns npatch x PATCH ints.
std::vector<int> build_patches(const FreeMap& m, std::vector<int>* verts = nullptr);

// local tables shared with the structured path (host_tables.cpp)
void element_matrices(const PhysParams& p, double h, double A[2][13][13], bool kw[2][13][13]);
struct LocalProlong {
    int t_f, fi, fj;   // fine DoF type and slot in fine units, relative to the coarse square
    int t_c, cI, cJ;   // coarse DoF type and slot, relative to the coarse square
    double w;
};
void local_prolongation_entries(std::vector<LocalProlong>& out);

// ---- device launches (sparse.hip) ----------------------------------------------------------------
// y = c z + a A x over the rows of a CSR matrix; x == nullptr: A x = 0; z == nullptr: z = 0.
// y may alias z, not x.
void launch_csr_mv(int rows, const int* ptr, const int* col, const double* val, const double* x, const double* z,
                   double* y, double a, double c, hipStream_t st);
// val[e] = val0[e] + sum_{q in [kptr[e], kptr[e+1])} kcoef[q] kinv[ktri[q]]
void launch_csr_assemble(int nnz, const double* val0, const int* kptr, const int* ktri, const double* kcoef,
                         const double* kinv, double* val, hipStream_t st);
// per-triangle 1/K of the 2 n^2 triangles: mode 0 from K (K == nullptr: the scalar Ks), mode 1
// from theta = ln K (1/K = exp(-theta))
void launch_kinv_flat(long long ntri, const double* K, double Ks, int mode, double* kinv, hipStream_t st);
// 1/K of the 2 nc^2 coarse triangles: the mean of the four children's (fine mesh 2 nc)
void launch_kinv_coarsen_flat(int nc, const double* kf, double* kc, hipStream_t st);
// inverse of every shifted patch matrix V_l A V_l^T + shift S (S = +1 on the displacement and
// Darcy slots, -1 on the pressure slots; identity on absent slots), column-major 20 x 20 per
// patch; *status = 1 if a pivot vanished
void launch_patch_inverse(int np, const int* slots, const int* ptr, const int* col, const double* val, double shift,
                          double* inv, int* status, hipStream_t st);
// y[p][a] = sum_b inv_p[a][b] r[slots[p][b]] (0 on absent slots)
void launch_patch_apply(int np, const int* slots, const double* inv, const double* r, double* y, hipStream_t st);
// xout[d] = x[d] + omega wgt[d] sum_{q in [dptr[d], dptr[d+1])} y[dlist[q]]  (x == nullptr: 0;
// xout may alias x)
void launch_patch_gather(int N, const int* dptr, const int* dlist, const double* y, const double* wgt, double omega,
                         const double* x, double* xout, hipStream_t st);
// row-major dense copy of a CSR matrix (N x N)
void launch_csr_to_dense(int N, const int* ptr, const int* col, const double* val, double* D, hipStream_t st);
// one colour step of multiplicative Vanka on explicit inverses: for the npc patches plist[k] of
// one colour (no two share a DoF), x[slots[p][a]] += omega (A_p^{-1} V_p r)[a]
void launch_patch_apply_add(int npc, const int* plist, const int* slots, const double* inv, const double* r,
                            double omega, double* x, hipStream_t st);
// the same colour step fused with its residual, in place: for the colour's patches (vertices of
// one colour share no mesh edge, so a patch's residual rows read no DoF another patch of the
// colour writes), r = b - A x on the patch rows, then x += omega A_p^{-1} r; xzero: the iterate
// is zero (r = b; x is not read: the colour's DoFs are assigned, and the nz DoFs of zlist, those
// no patch of the colour holds, are set to zero in the same launch).  crow[k * PATCH + a]: the
// DoF of slot a of the colour's k-th patch (-1 absent), cbeg / cend its CSR row bounds (plist[k]
// the patch, for its inverse)
void launch_colour_step(int npc, const int* plist, const int* crow, const int* cbeg, const int* cend,
                        const double* inv, const int* col, const double* val, const double* b, double* x,
                        double omega, bool xzero, hipStream_t st, const int* zlist = nullptr, int nz = 0);
// per-triangle 1/K of a level of the padded layout (two planes) in the flat triangle order
void launch_kinv_unpad(const Layout& L, const double* kinv_padded, double* flat, hipStream_t st);

}  // namespace biot
