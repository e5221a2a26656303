// Host-side construction of the constant tables of the solver: the stencil of the
// rediscretized RQ Biot operator (from the element matrices), the gather tables of the
// block prolongation, and the per-class data of the Vanka patch solves.
//
// Paper: Sec. 2.1 (spaces, block_form), Sec. 2.3 (block_form_rq), Appendix A
// (A_u^RQ = 2 mu A_eps + lambda B_u^T M_p^-1 B_u), Sec. 3 (eq. block_interp, R = P^T),
// Sec. 3.1 (divergence-preserving P_u), Sec. 3.2.1 (vertex patches).
#include "common.h"
#include "sparse.h"
#include "structure.h"

#include <array>
#include <cmath>
#include <map>
#include <stdexcept>
#include <tuple>

namespace biot {

namespace {

struct V2 {
    double x, y;
};
inline V2 operator+(V2 a, V2 b) { return {a.x + b.x, a.y + b.y}; }
inline V2 operator-(V2 a, V2 b) { return {a.x - b.x, a.y - b.y}; }
inline V2 operator*(double s, V2 a) { return {s * a.x, s * a.y}; }
inline double dot(V2 a, V2 b) { return a.x * b.x + a.y * b.y; }

// Global edge kinds and their unit normals.
enum EdgeKind { EH = 0, EV = 1, ED = 2 };
inline V2 edge_normal(int kind) {
    const double s = 1.0 / std::sqrt(2.0);
    if (kind == EH) return {0.0, 1.0};
    if (kind == EV) return {1.0, 0.0};
    return {s, s};
}

// Identify the edge between two lattice points (integer coordinates in units of the
// mesh size): kind and anchoring slot.
inline void edge_of(V2 a, V2 b, int& kind, int& si, int& sj) {
    int ax = (int)std::lround(a.x), ay = (int)std::lround(a.y);
    int bx = (int)std::lround(b.x), by = (int)std::lround(b.y);
    if (ay == by) {
        kind = EH;
        si = std::min(ax, bx);
        sj = ay;
    } else if (ax == bx) {
        kind = EV;
        si = ax;
        sj = std::min(ay, by);
    } else {
        kind = ED;
        si = std::min(ax, bx);
        sj = std::min(ay, by);
    }
}

// ---- one triangle of the square (0, 0): geometry, local DoF map, element matrices -----
struct Tri {
    V2 X[3];               // vertices (units of h), counter-clockwise
    int ekind[3];          // kind of the edge opposite vertex k
    int esi[3], esj[3];    // its anchoring slot
    // local DoFs: 0..2 ux(v), 3..5 uy(v), 6..8 bubble(e), 9..11 rt0(e), 12 p
    int type[13], di[13], dj[13];
};

Tri make_tri(bool upper) {
    Tri t;
    if (!upper) {
        t.X[0] = {0, 0}; t.X[1] = {1, 0}; t.X[2] = {0, 1};
    } else {
        t.X[0] = {1, 0}; t.X[1] = {1, 1}; t.X[2] = {0, 1};
    }
    for (int k = 0; k < 3; ++k) {
        edge_of(t.X[(k + 1) % 3], t.X[(k + 2) % 3], t.ekind[k], t.esi[k], t.esj[k]);
        int vx = (int)std::lround(t.X[k].x), vy = (int)std::lround(t.X[k].y);
        t.type[k] = T_UX; t.di[k] = vx; t.dj[k] = vy;
        t.type[3 + k] = T_UY; t.di[3 + k] = vx; t.dj[3 + k] = vy;
        const int bt[3] = {T_BH, T_BV, T_BD}, wt[3] = {T_WH, T_WV, T_WD};
        t.type[6 + k] = bt[t.ekind[k]]; t.di[6 + k] = t.esi[k]; t.dj[6 + k] = t.esj[k];
        t.type[9 + k] = wt[t.ekind[k]]; t.di[9 + k] = t.esi[k]; t.dj[9 + k] = t.esj[k];
    }
    t.type[12] = upper ? T_PU : T_PL;
    t.di[12] = 0;
    t.dj[12] = 0;
    return t;
}

// Element matrices of a triangle scaled by h (Sec. 2.1 / 2.3 forms, exact midpoint rule).
struct ElemMats {
    double area;
    double Keps[9][9];  // int eps(phi_i) : eps(phi_j)
    double g[9];        // int_T div phi_i
    double Mw[3][3];    // int psi_k . psi_l   (K = mu_f = 1)
    double Bw[3];       // -int_T div psi_k
};

ElemMats element_mats(const Tri& t, double h) {
    ElemMats E{};
    V2 X[3];
    for (int k = 0; k < 3; ++k) X[k] = h * t.X[k];
    V2 e1 = X[1] - X[0], e2 = X[2] - X[0];
    double det = e1.x * e2.y - e1.y * e2.x;  // 2|T| > 0
    E.area = 0.5 * det;
    V2 gl[3];
    double len[3], sig[3];
    V2 nrm[3];
    for (int k = 0; k < 3; ++k) {
        V2 a = X[(k + 1) % 3], b = X[(k + 2) % 3], e = b - a;
        gl[k] = {-e.y / det, e.x / det};  // grad of barycentric coordinate k
        len[k] = std::sqrt(dot(e, e));
        nrm[k] = edge_normal(t.ekind[k]);
        sig[k] = dot(nrm[k], 0.5 * (a + b) - X[k]) > 0 ? 1.0 : -1.0;
    }
    const double qb[3][3] = {{0, .5, .5}, {.5, 0, .5}, {.5, .5, 0}};
    const double w = E.area / 3.0;
    for (int q = 0; q < 3; ++q) {
        const double* be = qb[q];
        double G[9][2][2] = {};
        for (int a = 0; a < 3; ++a) {
            G[a][0][0] = gl[a].x; G[a][0][1] = gl[a].y;
            G[3 + a][1][0] = gl[a].x; G[3 + a][1][1] = gl[a].y;
        }
        for (int k = 0; k < 3; ++k) {
            int p = (k + 1) % 3, r = (k + 2) % 3;
            V2 gs = 4.0 * (be[r] * gl[p] + be[p] * gl[r]);
            G[6 + k][0][0] = nrm[k].x * gs.x; G[6 + k][0][1] = nrm[k].x * gs.y;
            G[6 + k][1][0] = nrm[k].y * gs.x; G[6 + k][1][1] = nrm[k].y * gs.y;
        }
        double eps[9][2][2];
        for (int i = 0; i < 9; ++i)
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d) eps[i][c][d] = 0.5 * (G[i][c][d] + G[i][d][c]);
        for (int i = 0; i < 9; ++i) {
            E.g[i] += w * (G[i][0][0] + G[i][1][1]);
            for (int j = 0; j < 9; ++j) {
                double s = 0;
                for (int c = 0; c < 2; ++c)
                    for (int d = 0; d < 2; ++d) s += eps[i][c][d] * eps[j][c][d];
                E.Keps[i][j] += w * s;
            }
        }
        V2 xq = be[0] * X[0] + be[1] * X[1] + be[2] * X[2];
        V2 psi[3];
        for (int k = 0; k < 3; ++k) psi[k] = (sig[k] * len[k] / (2.0 * E.area)) * (xq - X[k]);
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) E.Mw[k][l] += w * dot(psi[k], psi[l]);
    }
    for (int k = 0; k < 3; ++k) E.Bw[k] = -sig[k] * len[k];
    return E;
}

// 13 x 13 local matrix of the RQ Biot system; kw marks the K-dependent (RT0 mass) part.
void local_matrix(const ElemMats& E, const PhysParams& p, double A[13][13], bool kw[13][13]) {
    for (int i = 0; i < 13; ++i)
        for (int j = 0; j < 13; ++j) {
            A[i][j] = 0;
            kw[i][j] = false;
        }
    for (int i = 0; i < 9; ++i) {
        for (int j = 0; j < 9; ++j)
            A[i][j] = 2.0 * p.mu * E.Keps[i][j] + p.lambda * E.g[i] * E.g[j] / E.area;
        A[i][12] = A[12][i] = -p.alpha * E.g[i];
    }
    for (int k = 0; k < 3; ++k) {
        for (int l = 0; l < 3; ++l) {
            A[9 + k][9 + l] = p.tau * p.mu_f * E.Mw[k][l];
            kw[9 + k][9 + l] = true;
        }
        A[9 + k][12] = A[12][9 + k] = p.tau * E.Bw[k];
    }
    A[12][12] = -p.inv_M * E.area;
}

}  // namespace

void element_matrices(const PhysParams& p, double h, double A[2][13][13], bool kw[2][13][13]) {
    for (int u = 0; u < 2; ++u) local_matrix(element_mats(make_tri(u == 1), h), p, A[u], kw[u]);
}

void build_stencil_coef(const PhysParams& p, double h, double* coef) {
    Tri tris[2] = {make_tri(false), make_tri(true)};
    double A[2][13][13];
    bool kw[2][13][13];
    for (int u = 0; u < 2; ++u) {
        local_matrix(element_mats(tris[u], h), p, A[u], kw[u]);
        for (int k = 0; k < 13; ++k) {
            const LDof d = ldof(u, k);
            if (d.t != tris[u].type[k] || d.di != tris[u].di[k] || d.dj != tris[u].dj[k])
                throw std::runtime_error("local DoF map mismatch");
            for (int k2 = 0; k2 < 13; ++k2)
                if (!lcoupled(k, k2) && A[u][k][k2] != 0.0) throw std::runtime_error("coupling outside structure");
        }
    }
    for (int q = 0; q < NSTENCIL; ++q) coef[q] = 0.0;
    for (int t = 0; t < NTYPES; ++t)
        for (int sj = -1; sj <= 0; ++sj)
            for (int si = -1; si <= 0; ++si)
                for (int u = 0; u < 2; ++u)
                    for (int k = 0; k < 13; ++k) {
                        const LDof r = ldof(u, k);
                        if (r.t != t || si + r.di != 0 || sj + r.dj != 0) continue;
                        for (int k2 = 0; k2 < 13; ++k2) {
                            if (!lcoupled(k, k2)) continue;
                            const SEnt en = stencil_key(u, si, sj, k2, lkdep(k, k2));
                            int found = -1;
                            for (int q = 0; q < SST.n[t]; ++q)
                                if (sent_eq(SST.e[t][q], en)) found = q;
                            if (found < 0) throw std::runtime_error("stencil structure mismatch");
                            coef[SST.off[t] + found] += A[u][k][k2];
                        }
                    }
}

std::vector<StencilEntry> build_stencil(const PhysParams& p, double h) {
    std::vector<double> coef(NSTENCIL);
    build_stencil_coef(p, h, coef.data());
    std::vector<StencilEntry> out;
    for (int t = 0; t < NTYPES; ++t)
        for (int q = 0; q < SST.n[t]; ++q) {
            const SEnt& en = SST.e[t][q];
            StencilEntry e{};
            e.out_t = (int8_t)t;
            e.in_t = (int8_t)en.in;
            e.di = (int8_t)en.di;
            e.dj = (int8_t)en.dj;
            e.ktri = (int8_t)en.kt;
            e.kdi = (int8_t)en.kdi;
            e.kdj = (int8_t)en.kdj;
            e.coef = coef[SST.off[t] + q];
            out.push_back(e);
        }
    return out;
}

// ---- prolongation tables (Sec. 3, 3.1) ------------------------------------------------------
namespace {

// Coarse triangle of the coarse square (0,0), in fine units (coarse h = 2).
struct CTri {
    V2 X[3];
    int ekind[3];
    int type[13], dI[13], dJ[13];  // coarse local DoF -> coarse type and coarse slot
    double sig[3], len[3], area;
};

CTri make_ctri(bool upper) {
    Tri t = make_tri(upper);
    CTri c;
    for (int k = 0; k < 3; ++k) {
        c.X[k] = 2.0 * t.X[k];
        c.ekind[k] = t.ekind[k];
    }
    for (int k = 0; k < 13; ++k) {
        c.type[k] = t.type[k];
        c.dI[k] = t.di[k];
        c.dJ[k] = t.dj[k];
    }
    V2 e1 = c.X[1] - c.X[0], e2 = c.X[2] - c.X[0];
    c.area = 0.5 * (e1.x * e2.y - e1.y * e2.x);
    for (int k = 0; k < 3; ++k) {
        V2 a = c.X[(k + 1) % 3], b = c.X[(k + 2) % 3];
        c.len[k] = std::sqrt(dot(b - a, b - a));
        c.sig[k] = dot(edge_normal(c.ekind[k]), 0.5 * (a + b) - c.X[k]) > 0 ? 1.0 : -1.0;
    }
    return c;
}

// Value of the 9 coarse displacement basis functions at barycentric point be.
void coarse_u_values(const CTri& c, const double be[3], V2 out[9]) {
    for (int a = 0; a < 3; ++a) {
        out[a] = {be[a], 0.0};
        out[3 + a] = {0.0, be[a]};
    }
    for (int k = 0; k < 3; ++k) {
        int p = (k + 1) % 3, q = (k + 2) % 3;
        out[6 + k] = (4.0 * be[p] * be[q]) * edge_normal(c.ekind[k]);
    }
}

struct Bary {
    double b[3];
};
Bary corner(int k) {
    Bary r{{0, 0, 0}};
    r.b[k] = 1;
    return r;
}
Bary midb(int a, int b) {
    Bary r{{0, 0, 0}};
    r.b[a] = r.b[b] = 0.5;
    return r;
}
V2 pos(const CTri& c, const Bary& b) { return b.b[0] * c.X[0] + b.b[1] * c.X[1] + b.b[2] * c.X[2]; }

struct RawP {
    int t_f, fi, fj, t_c, cI, cJ;
    double w;
};

void add_raw(std::vector<RawP>& v, int t_f, int fi, int fj, int t_c, int cI, int cJ, double w) {
    v.push_back({t_f, fi, fj, t_c, cI, cJ, w});
}

void local_prolongation(bool upper, std::vector<RawP>& raw) {
    CTri c = make_ctri(upper);
    const int bt[3] = {T_BH, T_BV, T_BD}, wt[3] = {T_WH, T_WV, T_WD};
    // fine vertices: corners and edge midpoints of the coarse triangle
    Bary fv[6] = {corner(0), corner(1), corner(2), midb(1, 2), midb(0, 2), midb(0, 1)};
    for (auto& b : fv) {
        V2 u[9];
        coarse_u_values(c, b.b, u);
        V2 x = pos(c, b);
        int fi = (int)std::lround(x.x), fj = (int)std::lround(x.y);
        for (int f = 0; f < 9; ++f) {
            add_raw(raw, T_UX, fi, fj, c.type[f], c.dI[f], c.dJ[f], u[f].x);
            add_raw(raw, T_UY, fi, fj, c.type[f], c.dI[f], c.dJ[f], u[f].y);
        }
    }
    // canonical bubble coefficient on a fine edge [a, b]: (u(m) - (u(a)+u(b))/2) . n_e
    auto bubble_coef = [&](const Bary& a, const Bary& b, double coef[9], int& kind, int& si,
                           int& sj, double& L) {
        Bary m{{0.5 * (a.b[0] + b.b[0]), 0.5 * (a.b[1] + b.b[1]), 0.5 * (a.b[2] + b.b[2])}};
        V2 ua[9], ub[9], um[9];
        coarse_u_values(c, a.b, ua);
        coarse_u_values(c, b.b, ub);
        coarse_u_values(c, m.b, um);
        V2 xa = pos(c, a), xb = pos(c, b);
        edge_of(xa, xb, kind, si, sj);
        V2 ne = edge_normal(kind);
        L = std::sqrt(dot(xb - xa, xb - xa));
        for (int f = 0; f < 9; ++f) coef[f] = dot(um[f] - 0.5 * (ua[f] + ub[f]), ne);
    };
    // half edges of the coarse edges
    for (int k = 0; k < 3; ++k) {
        int p = (k + 1) % 3, q = (k + 2) % 3;
        Bary ends[2][2] = {{corner(p), midb(p, q)}, {midb(p, q), corner(q)}};
        for (auto& e : ends) {
            double cf[9], L;
            int kind, si, sj;
            bubble_coef(e[0], e[1], cf, kind, si, sj, L);
            for (int f = 0; f < 9; ++f) add_raw(raw, bt[kind], si, sj, c.type[f], c.dI[f], c.dJ[f], cf[f]);
        }
    }
    // corner children: zero net normal flux (Sec. 3.1, eq. divfreefine)
    for (int k = 0; k < 3; ++k) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        Bary vv[3] = {corner(k), midb(k, a), midb(k, b)};
        V2 cen = (1.0 / 3.0) * (pos(c, vv[0]) + pos(c, vv[1]) + pos(c, vv[2]));
        double flux[9] = {0};
        int ikind = -1, isi = 0, isj = 0;
        double isig = 0, ilen = 0;
        for (int s = 0; s < 3; ++s) {
            const Bary& ba = vv[s];
            const Bary& bb = vv[(s + 1) % 3];
            V2 xa = pos(c, ba), xb = pos(c, bb);
            int kind, si, sj;
            edge_of(xa, xb, kind, si, sj);
            V2 ne = edge_normal(kind);
            double L = std::sqrt(dot(xb - xa, xb - xa));
            double sg = dot(ne, 0.5 * (xa + xb) - cen) > 0 ? 1.0 : -1.0;
            V2 ua[9], ub[9];
            coarse_u_values(c, ba.b, ua);
            coarse_u_values(c, bb.b, ub);
            for (int f = 0; f < 9; ++f) flux[f] += L * dot(0.5 * (ua[f] + ub[f]), sg * ne);
            bool interior = (s == 1);  // edge between the two midpoints
            if (interior) {
                ikind = kind; isi = si; isj = sj; isig = sg; ilen = L;
            } else {
                double cf[9], L2;
                int k2, s2i, s2j;
                bubble_coef(ba, bb, cf, k2, s2i, s2j, L2);
                for (int f = 0; f < 9; ++f) flux[f] += sg * cf[f] * (2.0 / 3.0) * L;
            }
        }
        for (int f = 0; f < 9; ++f) {
            double ci = -flux[f] / (isig * (2.0 / 3.0) * ilen);
            add_raw(raw, bt[ikind], isi, isj, c.type[f], c.dI[f], c.dJ[f], ci);
        }
    }
    // P_w: normal component of the coarse RT0 functions at each fine edge midpoint
    std::vector<std::pair<Bary, Bary>> fe;
    for (int k = 0; k < 3; ++k) {
        int p = (k + 1) % 3, q = (k + 2) % 3;
        fe.push_back({corner(p), midb(p, q)});
        fe.push_back({midb(p, q), corner(q)});
    }
    fe.push_back({midb(0, 1), midb(1, 2)});
    fe.push_back({midb(1, 2), midb(0, 2)});
    fe.push_back({midb(0, 2), midb(0, 1)});
    for (auto& e : fe) {
        V2 xa = pos(c, e.first), xb = pos(c, e.second), xm = 0.5 * (xa + xb);
        int kind, si, sj;
        edge_of(xa, xb, kind, si, sj);
        V2 ne = edge_normal(kind);
        for (int k = 0; k < 3; ++k) {
            V2 psi = (c.sig[k] * c.len[k] / (2.0 * c.area)) * (xm - c.X[k]);
            add_raw(raw, wt[kind], si, sj, c.type[9 + k], c.dI[9 + k], c.dJ[9 + k], dot(psi, ne));
        }
    }
    // P_p: the four children take the parent value
    Bary ch[4][3] = {{corner(0), midb(0, 1), midb(0, 2)},
                     {corner(1), midb(1, 2), midb(0, 1)},
                     {corner(2), midb(0, 2), midb(1, 2)},
                     {midb(0, 1), midb(1, 2), midb(0, 2)}};
    for (auto& tr : ch) {
        V2 cen = (1.0 / 3.0) * (pos(c, tr[0]) + pos(c, tr[1]) + pos(c, tr[2]));
        int si = (int)std::floor(cen.x), sj = (int)std::floor(cen.y);
        bool up = (cen.x - si) + (cen.y - sj) > 1.0;
        add_raw(raw, up ? T_PU : T_PL, si, sj, c.type[12], c.dI[12], c.dJ[12], 1.0);
    }
}

}  // namespace

void build_prolong_weights(double* w) {
    std::vector<RawP> raw[2];
    local_prolongation(false, raw[0]);
    local_prolongation(true, raw[1]);
    for (int q = 0; q < NPWEIGHTS; ++q) w[q] = 0.0;
    for (int t = 0; t < NTYPES; ++t)
        for (int pj = 0; pj < 2; ++pj)
            for (int pi = 0; pi < 2; ++pi) {
                const int u = fine_tri(t, pi, pj);
                for (int q = 0; q < fcount(t); ++q) {
                    const LDof c = ldof(u, ffirst(t) + q);
                    for (auto& r : raw[u])
                        if (r.t_f == t && r.fi == pi && r.fj == pj && r.t_c == c.t && r.cI == c.di && r.cJ == c.dj)
                            w[widx(t, pi, pj, q)] = r.w;
                }
            }
}

void local_prolongation_entries(std::vector<LocalProlong>& out) {
    std::vector<RawP> raw;
    local_prolongation(false, raw);
    local_prolongation(true, raw);
    out.clear();
    for (auto& r : raw) out.push_back({r.t_f, r.fi, r.fj, r.t_c, r.cI, r.cJ, r.w});
}

void build_transfer_tables(std::vector<ProlongEntry>& pro, std::vector<RestrictEntry>& res) {
    std::vector<RawP> raw;
    local_prolongation(false, raw);
    local_prolongation(true, raw);
    std::map<std::array<int, 6>, double> uniq;
    for (auto& r : raw) {
        if (std::fabs(r.w) < 1e-14) continue;
        int pi = ((r.fi % 2) + 2) % 2, pj = ((r.fj % 2) + 2) % 2;
        int a = (r.fi - pi) / 2, b = (r.fj - pj) / 2;
        std::array<int, 6> key{r.t_f, pi, pj, r.t_c, r.cI - a, r.cJ - b};
        auto it = uniq.find(key);
        if (it == uniq.end()) {
            uniq[key] = r.w;
        } else if (std::fabs(it->second - r.w) > 1e-12) {
            throw std::runtime_error("inconsistent prolongation weights");
        }
    }
    pro.clear();
    res.clear();
    for (auto& kv : uniq) {
        ProlongEntry e{};
        e.t_f = (int8_t)kv.first[0]; e.pi = (int8_t)kv.first[1]; e.pj = (int8_t)kv.first[2];
        e.t_c = (int8_t)kv.first[3]; e.dI = (int8_t)kv.first[4]; e.dJ = (int8_t)kv.first[5];
        e.w = kv.second;
        pro.push_back(e);
        RestrictEntry r{};
        r.t_c = e.t_c;
        r.t_f = e.t_f;
        r.di = (int8_t)(e.pi - 2 * e.dI);
        r.dj = (int8_t)(e.pj - 2 * e.dJ);
        r.w = e.w;
        res.push_back(r);
    }
    // group by output type (stable order inside each type)
    std::stable_sort(pro.begin(), pro.end(), [](const ProlongEntry& a, const ProlongEntry& b) {
        return std::make_tuple(a.t_f, a.pi, a.pj) < std::make_tuple(b.t_f, b.pi, b.pj);
    });
    std::stable_sort(res.begin(), res.end(),
                     [](const RestrictEntry& a, const RestrictEntry& b) { return a.t_c < b.t_c; });
}

// ---- Vanka patch classes ------------------------------------------------------------------------
namespace {

bool invert_dense(int N, const double* A, double* Inv) {
    std::vector<double> M(A, A + N * N);
    for (int i = 0; i < N * N; ++i) Inv[i] = 0;
    for (int i = 0; i < N; ++i) Inv[i * N + i] = 1;
    for (int c = 0; c < N; ++c) {
        int piv = c;
        for (int r = c + 1; r < N; ++r)
            if (std::fabs(M[r * N + c]) > std::fabs(M[piv * N + c])) piv = r;
        if (M[piv * N + c] == 0.0) return false;
        if (piv != c)
            for (int k = 0; k < N; ++k) {
                std::swap(M[piv * N + k], M[c * N + k]);
                std::swap(Inv[piv * N + k], Inv[c * N + k]);
            }
        double d = 1.0 / M[c * N + c];
        for (int k = 0; k < N; ++k) {
            M[c * N + k] *= d;
            Inv[c * N + k] *= d;
        }
        for (int r = 0; r < N; ++r) {
            if (r == c) continue;
            double f = M[r * N + c];
            if (f == 0.0) continue;
            for (int k = 0; k < N; ++k) {
                M[r * N + k] -= f * M[c * N + k];
                Inv[r * N + k] -= f * Inv[c * N + k];
            }
        }
    }
    return true;
}

// Dense patch matrix of vertex (i, j) from the stencil (K-dependent entries skipped).
void patch_matrix(const std::vector<StencilEntry>& st, int i, int j, int n, double P[PATCH][PATCH],
                  int present[PATCH]) {
    int t[PATCH], di[PATCH], dj[PATCH];
    for (int s = 0; s < PATCH; ++s) {
        patch_slot(s, t[s], di[s], dj[s]);
        present[s] = dof_free(t[s], i + di[s], j + dj[s], n) ? 1 : 0;
    }
    for (int a = 0; a < PATCH; ++a)
        for (int b = 0; b < PATCH; ++b) P[a][b] = 0;
    for (int a = 0; a < PATCH; ++a) {
        if (!present[a]) continue;
        for (auto& e : st) {
            if (e.out_t != t[a] || e.ktri >= 0) continue;
            for (int b = 0; b < PATCH; ++b) {
                if (!present[b] || e.in_t != t[b]) continue;
                if (e.di == di[b] - di[a] && e.dj == dj[b] - dj[a]) P[a][b] += e.coef;
            }
        }
    }
}

void vertex_of_class(int cls, int n, int& i, int& j) {
    int ci = cls % 3, cj = cls / 3;
    i = ci == 0 ? 0 : (ci == 1 ? n / 2 : n);
    j = cj == 0 ? 0 : (cj == 1 ? n / 2 : n);
}

}  // namespace

void build_patch_classes(const std::vector<StencilEntry>& st, int n, PatchClass cls[9],
                         std::vector<WEntry>& wentries) {
    for (int c = 0; c < 9; ++c) {
        int vi, vj;
        vertex_of_class(c, n, vi, vj);
        double P[PATCH][PATCH];
        int pres[PATCH];
        patch_matrix(st, vi, vj, n, P, pres);
        bool keep = false;
        for (int s = 0; s < 14; ++s) keep = keep || pres[s];
        PatchClass& pc = cls[c];
        for (int s = 0; s < PATCH; ++s) {
            pc.present[s] = keep ? pres[s] : 0;
            pc.weight[s] = 0;
        }
        double A[64], Ainv[64];
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b)
                A[a * 8 + b] = (pc.present[a] && pc.present[b]) ? P[a][b] : (a == b ? 1.0 : 0.0);
        if (!invert_dense(8, A, Ainv)) throw SingularError{"singular displacement patch block"};
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) pc.Ainv[a][b] = Ainv[a * 8 + b];
        double Bh[6][8];
        for (int q = 0; q < 6; ++q)
            for (int a = 0; a < 8; ++a)
                Bh[q][a] = (pc.present[14 + q] && pc.present[a]) ? P[14 + q][a] : 0.0;
        for (int a = 0; a < 8; ++a)
            for (int q = 0; q < 6; ++q) {
                double s = 0;
                for (int b = 0; b < 8; ++b) s += pc.Ainv[a][b] * Bh[q][b];
                pc.H[a][q] = s;
            }
        for (int q1 = 0; q1 < 6; ++q1)
            for (int q2 = 0; q2 < 6; ++q2) {
                double s = 0;
                for (int a = 0; a < 8; ++a) s += Bh[q1][a] * pc.H[a][q2];
                pc.G[q1][q2] = s;
            }
        for (int q = 0; q < 6; ++q) {
            for (int a = 0; a < 6; ++a)
                pc.Q[q][a] = (pc.present[14 + q] && pc.present[8 + a]) ? P[14 + q][8 + a] : 0.0;
            pc.c[q] = pc.present[14 + q] ? -P[14 + q][14 + q] : 0.0;
        }
    }
    // w-w entries of an interior patch, tagged with the star triangle of their 1/K
    wentries.clear();
    int vi = n / 2, vj = n / 2;
    int t[PATCH], di[PATCH], dj[PATCH];
    for (int s = 0; s < PATCH; ++s) patch_slot(s, t[s], di[s], dj[s]);
    for (int a = 8; a < 14; ++a)
        for (int b = 8; b < 14; ++b)
            for (auto& e : st) {
                if (e.ktri < 0 || e.out_t != t[a] || e.in_t != t[b]) continue;
                if (e.di != di[b] - di[a] || e.dj != dj[b] - dj[a]) continue;
                int tdi = di[a] + e.kdi, tdj = dj[a] + e.kdj, k = -1;
                for (int kk = 0; kk < 6; ++kk) {
                    int ut, sdi, sdj;
                    star_tri(kk, ut, sdi, sdj);
                    if (ut == e.ktri && sdi == tdi && sdj == tdj) k = kk;
                }
                if (k < 0) throw std::runtime_error("RT0 mass entry outside the vertex star");
                WEntry w{};
                w.a = (int8_t)(a - 8);
                w.b = (int8_t)(b - 8);
                w.k = (int8_t)k;
                w.coef = e.coef;
                wentries.push_back(w);
            }
    (void)vi;
    (void)vj;
}

void build_upatch_classes(const std::vector<StencilEntry>& st, int n, UPatchClass cls[9]) {
    for (int c = 0; c < 9; ++c) {
        int vi, vj;
        vertex_of_class(c, n, vi, vj);
        double P[PATCH][PATCH];
        int pres[PATCH];
        patch_matrix(st, vi, vj, n, P, pres);
        bool keep = false;
        for (int s = 0; s < 8; ++s) keep = keep || pres[s];
        UPatchClass& uc = cls[c];
        for (int s = 0; s < 8; ++s) {
            uc.present[s] = keep ? pres[s] : 0;
            uc.weight[s] = 0;
        }
        double A[64], Ainv[64];
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b)
                A[a * 8 + b] = (uc.present[a] && uc.present[b]) ? P[a][b] : (a == b ? 1.0 : 0.0);
        if (!invert_dense(8, A, Ainv)) throw SingularError{"singular displacement patch block"};
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) uc.Ainv[a][b] = Ainv[a * 8 + b];
    }
}

}  // namespace biot
