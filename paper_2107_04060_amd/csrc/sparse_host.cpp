// Host-side tables of the general-boundary path: the free-DoF numbering under a set of
// boundary conditions, the CSR pattern of the rediscretized operator with its assembly lists,
// the CSR block prolongation and the 20-slot vertex patches.
//
// Paper: Sec. 2.1 (spaces, block_form), Sec. 2.3 (block_form_rq: the element matrices are the
// structured path's), Sec. 3 (eq. block_interp, R = P^T), Sec. 3.1 (divergence-preserving
// P_u: the local rules are the structured path's), Sec. 3.2.1 (vertex patches), Sec. 5
// (Terzaghi's problem: which DoFs its boundary conditions eliminate).
#include "sparse.h"
#include "structure.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

namespace biot {

namespace {

// entities of type t on the n x n mesh: extent of i and j, and the position of slot (i, j) in
// its block of the full numbering (-1 outside)
long long full_pos(int t, int i, int j, int n) {
    switch (t) {
        case T_UX: case T_UY:
            return (i < 0 || i > n || j < 0 || j > n) ? -1 : (long long)j * (n + 1) + i;
        case T_BH: case T_WH:
            return (i < 0 || i >= n || j < 0 || j > n) ? -1 : (long long)j * n + i;
        case T_BV: case T_WV:
            return (i < 0 || i > n || j < 0 || j >= n) ? -1 : (long long)j * (n + 1) + i;
        default:  // D edges, L and U triangles
            return (i < 0 || i >= n || j < 0 || j >= n) ? -1 : (long long)j * n + i;
    }
}

long long full_block(int t, int n) {
    switch (t) {
        case T_UX: case T_UY: return (long long)(n + 1) * (n + 1);
        case T_BH: case T_WH: case T_BV: case T_WV: return (long long)n * (n + 1);
        default: return (long long)n * n;
    }
}

void type_range(int t, int n, int& imax, int& jmax) {
    imax = (t == T_UX || t == T_UY || t == T_BV || t == T_WV) ? n : n - 1;
    jmax = (t == T_UX || t == T_UY || t == T_BH || t == T_WH) ? n : n - 1;
}

// is the existing DoF (t, i, j) free under bc?
bool is_free(int bc, int t, int i, int j, int n) {
    if (bc == BC_DIRICHLET) return dof_free(t, i, j, n);
    // Terzaghi: fixed face x = 1 (i = n) eliminates u and the normal components of its edges;
    // the rollers y = 0, y = n eliminate u_y and the normal components (bubble, RT0) of their
    // horizontal edges; the loaded, drained face x = 0 keeps everything
    switch (t) {
        case T_UX: return i < n;
        case T_UY: return i < n && j > 0 && j < n;
        case T_BH: case T_WH: return j > 0 && j < n;
        case T_BV: case T_WV: return i < n;
        default: return true;
    }
}

}  // namespace

int FreeMap::index(int t, int i, int j) const {
    const long long p = full_pos(t, i, j, n);
    return p < 0 ? -1 : free_of_full[(size_t)(full_off[t] + p)];
}

FreeMap make_free_map(int n, int bc) {
    if (bc != BC_DIRICHLET && bc != BC_TERZAGHI) throw std::invalid_argument("unknown boundary conditions");
    FreeMap m;
    m.n = n;
    m.bc = bc;
    m.full_off[0] = 0;
    for (int t = 0; t < NTYPES; ++t) m.full_off[t + 1] = m.full_off[t] + full_block(t, n);
    m.free_of_full.assign((size_t)m.full_off[NTYPES], -1);
    int next = 0;
    for (int t = 0; t < NTYPES; ++t) {
        int imax, jmax;
        type_range(t, n, imax, jmax);
        for (int j = 0; j <= jmax; ++j)
            for (int i = 0; i <= imax; ++i)
                if (is_free(bc, t, i, j, n)) {
                    m.free_of_full[(size_t)(m.full_off[t] + full_pos(t, i, j, n))] = next++;
                    ++m.block[t];
                }
    }
    m.N = next;
    m.n_u = (int)(m.block[T_UX] + m.block[T_UY] + m.block[T_BH] + m.block[T_BV] + m.block[T_BD]);
    m.n_w = (int)(m.block[T_WH] + m.block[T_WV] + m.block[T_WD]);
    m.n_p = (int)(m.block[T_PL] + m.block[T_PU]);
    return m;
}

OperatorHost build_operator(const FreeMap& m, const PhysParams& p) {
    const int n = m.n;
    double A[2][13][13];
    bool kw[2][13][13];
    element_matrices(p, 1.0 / n, A, kw);
    // contributions (row, column, triangle or -1, value), one per coupled pair of every triangle
    struct Cb {
        int r, c, tri;
        double v;
    };
    std::vector<Cb> cb;
    cb.reserve((size_t)2 * n * n * 120);
    int g[13];
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            for (int u = 0; u < 2; ++u) {
                const int tri = u * n * n + j * n + i;
                for (int k = 0; k < 13; ++k) {
                    const LDof d = ldof(u, k);
                    g[k] = m.index(d.t, i + d.di, j + d.dj);
                }
                for (int k = 0; k < 13; ++k) {
                    if (g[k] < 0) continue;
                    for (int k2 = 0; k2 < 13; ++k2) {
                        if (g[k2] < 0) continue;
                        if (kw[u][k][k2])
                            cb.push_back({g[k], g[k2], tri, A[u][k][k2]});
                        else if (A[u][k][k2] != 0.0)
                            cb.push_back({g[k], g[k2], -1, A[u][k][k2]});
                    }
                }
            }
    std::stable_sort(cb.begin(), cb.end(), [](const Cb& a, const Cb& b) {
        return a.r != b.r ? a.r < b.r : (a.c != b.c ? a.c < b.c : a.tri < b.tri);
    });
    OperatorHost op;
    op.A.rows = op.A.cols = m.N;
    op.A.ptr.assign((size_t)m.N + 1, 0);
    op.kptr.push_back(0);
    for (size_t q = 0; q < cb.size();) {
        const int r = cb[q].r, c = cb[q].c;
        double v0 = 0.0;
        for (; q < cb.size() && cb[q].r == r && cb[q].c == c; ++q) {
            if (cb[q].tri < 0) {
                v0 += cb[q].v;
            } else {
                op.ktri.push_back(cb[q].tri);
                op.kcoef.push_back(cb[q].v);
            }
        }
        op.A.col.push_back(c);
        op.A.val.push_back(v0);
        op.kptr.push_back((int)op.ktri.size());
        ++op.A.ptr[(size_t)r + 1];
    }
    for (int r = 0; r < m.N; ++r) op.A.ptr[(size_t)r + 1] += op.A.ptr[r];
    return op;
}

CsrHost build_prolongation(const FreeMap& fine, const FreeMap& coarse) {
    if (fine.n != 2 * coarse.n || fine.bc != coarse.bc) throw std::invalid_argument("levels do not nest");
    std::vector<LocalProlong> loc;
    local_prolongation_entries(loc);
    struct E {
        int f, c;
        double w;
    };
    std::vector<E> e;
    const int nc = coarse.n;
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I < nc; ++I)
            for (const LocalProlong& r : loc) {
                if (std::fabs(r.w) < 1e-14) continue;
                const int f = fine.index(r.t_f, 2 * I + r.fi, 2 * J + r.fj);
                const int c = coarse.index(r.t_c, I + r.cI, J + r.cJ);
                if (f < 0 || c < 0) continue;
                e.push_back({f, c, r.w});
            }
    std::stable_sort(e.begin(), e.end(), [](const E& a, const E& b) { return a.f != b.f ? a.f < b.f : a.c < b.c; });
    CsrHost P;
    P.rows = fine.N;
    P.cols = coarse.N;
    P.ptr.assign((size_t)fine.N + 1, 0);
    for (size_t q = 0; q < e.size();) {
        const int f = e[q].f, c = e[q].c;
        const double w = e[q].w;
        // the coarse triangles sharing a fine DoF give it the same weight (the rules depend on
        // the trace on the shared coarse edge only)
        for (; q < e.size() && e[q].f == f && e[q].c == c; ++q)
            if (std::fabs(e[q].w - w) > 1e-12 * std::max(1.0, std::fabs(w)))
                throw std::runtime_error("inconsistent prolongation weight");
        P.col.push_back(c);
        P.val.push_back(w);
        ++P.ptr[(size_t)f + 1];
    }
    for (int r = 0; r < fine.N; ++r) P.ptr[(size_t)r + 1] += P.ptr[r];
    return P;
}

CsrHost csr_transpose(const CsrHost& a) {
    CsrHost t;
    t.rows = a.cols;
    t.cols = a.rows;
    t.ptr.assign((size_t)a.cols + 1, 0);
    for (int c : a.col) ++t.ptr[(size_t)c + 1];
    for (int r = 0; r < a.cols; ++r) t.ptr[(size_t)r + 1] += t.ptr[r];
    t.col.resize(a.col.size());
    t.val.resize(a.val.size());
    std::vector<int> fill(t.ptr.begin(), t.ptr.end() - 1);
    for (int r = 0; r < a.rows; ++r)            // rows in order: columns of t come out sorted
        for (int q = a.ptr[r]; q < a.ptr[(size_t)r + 1]; ++q) {
            const int d = fill[a.col[q]]++;
            t.col[d] = r;
            t.val[d] = a.val[q];
        }
    return t;
}

std::vector<int> build_patches(const FreeMap& m, std::vector<int>* verts) {
    const int n = m.n;
    std::vector<int> out;
    if (verts) verts->clear();
    for (int j = 0; j <= n; ++j)
        for (int i = 0; i <= n; ++i) {
            const int s[PATCH] = {
                m.index(T_UX, i, j),         m.index(T_UY, i, j),
                m.index(T_BH, i - 1, j),     m.index(T_BH, i, j),
                m.index(T_BV, i, j - 1),     m.index(T_BV, i, j),
                m.index(T_BD, i - 1, j),     m.index(T_BD, i, j - 1),
                m.index(T_WH, i - 1, j),     m.index(T_WH, i, j),
                m.index(T_WV, i, j - 1),     m.index(T_WV, i, j),
                m.index(T_WD, i - 1, j),     m.index(T_WD, i, j - 1),
                m.index(T_PL, i, j),         m.index(T_PL, i - 1, j),
                m.index(T_PL, i, j - 1),     m.index(T_PU, i - 1, j - 1),
                m.index(T_PU, i - 1, j),     m.index(T_PU, i, j - 1)};
            bool keep = false;
            for (int a = 0; a < 14; ++a) keep = keep || s[a] >= 0;
            if (keep) {
                out.insert(out.end(), s, s + PATCH);
                if (verts) verts->push_back(j * (n + 1) + i);
            }
        }
    return out;
}

}  // namespace biot
