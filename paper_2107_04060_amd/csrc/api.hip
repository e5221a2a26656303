// C ABI of the RQ Biot monolithic multigrid library (declared in include/biot_mg.h):
// context lifetime, hierarchy set-up, V-cycle and FGMRES orchestration on a HIP stream.
//
// Paper passages: Sec. 3 (V-cycle structure, rediscretization, R = P^T), Sec. 3.2
// (relaxation), Sec. 5.1 (FGMRES with one V-cycle as preconditioner, zero initial guess,
// direct coarsest solve).
#include "../../include/biot_mg.h"
#include "common.h"
#include "kernels.h"
#include "patch_solve.h"
#include "sparse.h"
#include "structure.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>

namespace biot {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// ---- device memory helper ---------------------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b) {
        release();
        if (b == 0) return;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            throw std::bad_alloc();
        }
        bytes = b;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

template <typename T>
static void upload(DevBuf& d, const std::vector<T>& h, hipStream_t st) {
    d.alloc(std::max<size_t>(1, h.size()) * sizeof(T));
    if (!h.empty()) BIOT_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

struct Level {
    int n = 0;
    double h = 0;
    Layout L{};
    Canon C{};
    std::vector<StencilEntry> st_host;
    int st_off_host[NTYPES + 1];
    DevBuf st, st_off;                  // stencil entry list (device; coarse matrix set-up)
    DevBuf coef64, coef32;              // stencil coefficients in structure.h order
    DevBuf minv64;                      // full patch inverses per vertex class, uniform K (9 x 20 x 20)
    DevBuf kinv64, kinv32;              // 2 planes each
    DevBuf cls64, wblk64;               // per-class elimination data, RT0 blocks (FP64)
    DevBuf cls32, wblk32;               // the same in FP32 (FP32 variable-K eliminations)
    bool patch32 = false;               // FP32 variable-K eliminations on this level
    DevBuf uinv64, uinv32;              // displacement-patch inverses (BSR), 9 x 8 x 8
    DevBuf bsrd64, bsrd32;              // BSR diagonal data, 5 planes
    DevBuf x64, b64, r64, t64, x2_64;   // FP64 work vectors (padded); x64 / x2_64: iterate pair
    DevBuf x32, b32, r32, x2_32;        // FP32 work vectors (padded)
    DevBuf bs64, bs32;                  // BSR scratch vector (padded)
    DevBuf sch64, sch32;                // BSR Schur sweeps (s, two pressure buffers) or CG (dp, r, z, p, q): 10 planes
    DevBuf cgred;                       // BSR Schur CG: partial sums and scalars (doubles)
    DevBuf fac64;                       // variable K: the factors of every vertex patch (PFAC planes)
    double cS = 0;                      // (1/M + alpha^2 / (lambda + mu)) |T| of this level
    template <typename T>
    LevelView<T> view() const;
};

template <>
LevelView<double> Level::view<double>() const {
    LevelView<double> v;
    v.L = L;
    v.kinv = kinv64.as<double>();
    v.coef = coef64.as<double>();
    v.cls = cls64.as<DevPatchClass<double>>();
    v.wblk = wblk64.as<double>();
    v.cls32 = cls32.as<DevPatchClass<float>>();
    v.wblk32 = wblk32.as<float>();
    v.patch32 = false;
    v.uinv = uinv64.as<double>();
    v.bsrd = bsrd64.as<double>();
    v.minv = minv64.as<double>();
    v.fac = fac64.as<double>();
    return v;
}
template <>
LevelView<float> Level::view<float>() const {
    LevelView<float> v;
    v.L = L;
    v.kinv = kinv32.as<float>();
    v.coef = coef32.as<float>();
    v.cls = cls64.as<DevPatchClass<double>>();
    v.wblk = wblk64.as<double>();
    v.cls32 = cls32.as<DevPatchClass<float>>();
    v.wblk32 = wblk32.as<float>();
    v.patch32 = patch32;
    v.uinv = uinv32.as<float>();
    v.bsrd = bsrd32.as<float>();
    v.minv = minv64.as<double>();
    v.fac = fac64.as<double>();
    return v;
}

// One level of the general-boundary path (sparse.h): the CSR operator with its assembly lists,
// the transfers to the next coarser level, the explicit Vanka patch inverses and work vectors,
// all in the compact free-DoF order of the level.
struct SpLevel {
    FreeMap map;
    int N = 0, nnz = 0, np = 0;
    DevBuf ptr, col, val, val0, kptr, ktri, kcoef;  // A_l (CSR) and its assembly lists
    DevBuf kinv;                                    // 2 n^2 per-triangle 1/K
    DevBuf pptr, pcol, pval;                        // P from the next coarser level (rows: this level)
    DevBuf rptr, rcol, rval;                        // R = P^T (rows: the next coarser level)
    DevBuf slots, inv, y, dptr, dlist, wgt;         // additive Vanka: patches, inverses, corrections,
                                                    // DoF -> (patch, slot) lists, weights D = 1/count
    DevBuf x, b, r;                                 // iterate, right-hand side, residual
    DevBuf clist;                                   // multiplicative Vanka: patches by colour
    std::vector<int> coff;                          // colour c: clist[coff[c] .. coff[c+1])
    DevBuf crow, cbeg, cend;                        // their slots' rows and CSR row bounds
    DevBuf zlist0;                                  // the DoFs outside colour 0's patches
    int nz0 = 0;
    std::vector<int> ptr_h;                         // CSR row pointer (host copy)
};

struct SpHier {
    int bc = 0;
    std::vector<std::unique_ptr<SpLevel>> lv;       // lv[0] after assembly; the rest after set-up
    int cN = 0;                                     // coarsest level: dense inverse
    DevBuf cA, cinv, ccol, cidx, status;
};

}  // namespace biot

using namespace biot;

struct biot_ctx {
    int n = 0;
    PhysParams phys{};
    double K_scalar = 1.0;
    bool K_uniform = true;                        // permeability is the scalar K_scalar
    bool have_hierarchy = false;
    biot_mg_opts opts{};
    std::vector<std::unique_ptr<Level>> levels;   // levels[0] always exists after assemble
                                                  // (structured path; empty with sp)
    std::unique_ptr<SpHier> sp;                   // general-boundary path (bc != Dirichlet)
    std::unique_ptr<SpHier> small;                // Dirichlet path: levels small_from .. L-1 on CSR
    int small_from = -1;                          // (opts.csr_below; FP64 Vanka only)
    // transfers: prolongation weights (structure.h)
    DevBuf pw64, pw32;
    // coarsest level
    int coarse_N = 0;
    DevBuf coarse_A, coarse_inv, coarse_col, coarse_idx, coarse_map, status;
    DevBuf kcheck;                    // status word of the permeability checks (one int)
    // local RT0 mass (K = 1) of L and U for the adjoint gradient
    DevBuf mloc;
    // kernel timing (instrumentation)
    bool prof_on = false;
    int prof_level = 0;
    std::vector<hipEvent_t> prof_ev[2];   // [0] Vanka, [1] residual: start/stop pairs
    size_t prof_used[2] = {0, 0};
    ~biot_ctx() {
        for (auto& v : prof_ev)
            for (auto e : v) (void)hipEventDestroy(e);
        if (hhost) (void)hipHostFree(hhost);
    }
    // Krylov workspace
    int krylov_m = 0;
    DevBuf V, Z, w, partial, hdev, ydev, bpad, xpad, canon_tmp;
    double* hhost = nullptr;          // mapped pinned mirror of the Gram-Schmidt results
    double* hhost_dev = nullptr;      // its device address
    std::vector<double> hwork;        // host Hessenberg, rotations and least-squares vectors
};

namespace biot {

static void check_stream_error() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw HipError{e, "kernel launch"};
}

// ---- per-level set-up ----------------------------------------------------------------------------
static void level_alloc(Level& lv, int n, hipStream_t st) {
    lv.n = n;
    lv.h = 1.0 / n;
    lv.L = make_layout(n);
    lv.C = make_canon(n);
    const size_t len = (size_t)lv.L.len;
    lv.kinv64.alloc(2 * lv.L.plane * sizeof(double));
    lv.kinv32.alloc(2 * lv.L.plane * sizeof(float));
    for (DevBuf* b : {&lv.x64, &lv.b64, &lv.r64, &lv.t64, &lv.x2_64}) {
        b->alloc(len * sizeof(double));
        launch_fill(b->as<double>(), lv.L.len, 0.0, st);
    }
}

static void level_stencil(Level& lv, const PhysParams& p, hipStream_t st) {
    lv.st_host = build_stencil(p, lv.h);
    std::stable_sort(lv.st_host.begin(), lv.st_host.end(),
                     [](const StencilEntry& a, const StencilEntry& b) { return a.out_t < b.out_t; });
    for (int t = 0; t <= NTYPES; ++t) lv.st_off_host[t] = 0;
    for (auto& e : lv.st_host) lv.st_off_host[e.out_t + 1]++;
    for (int t = 0; t < NTYPES; ++t) lv.st_off_host[t + 1] += lv.st_off_host[t];
    upload(lv.st, lv.st_host, st);
    std::vector<int> off(lv.st_off_host, lv.st_off_host + NTYPES + 1);
    upload(lv.st_off, off, st);
    std::vector<double> coef(NSTENCIL);
    build_stencil_coef(p, lv.h, coef.data());
    upload(lv.coef64, coef, st);
    std::vector<float> cf(coef.begin(), coef.end());
    upload(lv.coef32, cf, st);
}

template <typename T>
static std::vector<DevPatchClass<T>> convert_classes(const PatchClass* c) {
    std::vector<DevPatchClass<T>> out(9);
    for (int k = 0; k < 9; ++k) {
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) out[k].Ainv[a][b] = (T)c[k].Ainv[a][b];
        for (int a = 0; a < 8; ++a)
            for (int q = 0; q < 6; ++q) out[k].H[a][q] = (T)c[k].H[a][q];
        for (int q = 0; q < 6; ++q) {
            for (int r = 0; r < 6; ++r) {
                out[k].G[q][r] = (T)c[k].G[q][r];
                out[k].Q[q][r] = (T)c[k].Q[q][r];
            }
            out[k].c[q] = (T)c[k].c[q];
        }
        for (int s = 0; s < PATCH; ++s) out[k].present[s] = c[k].present[s];
    }
    return out;
}

template <typename T>
static std::vector<T> convert_uinv(const UPatchClass* c) {
    std::vector<T> out(9 * 64);
    for (int k = 0; k < 9; ++k)
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) out[(k * 8 + a) * 8 + b] = (T)c[k].Ainv[a][b];
    return out;
}

static void level_patch_data(Level& lv, bool uniform, double Kinv, hipStream_t st) {
    PatchClass cls[9];
    std::vector<WEntry> we;
    build_patch_classes(lv.st_host, lv.n, cls, we);
    std::vector<double> wblk(24, 0.0);
    for (auto& e : we) {
        bool placed = false;
        for (int p = 0; p < 2 && !placed; ++p)
            for (int q = 0; q < 2 && !placed; ++q)
                if (star_wpair(e.k, p) == e.a && star_wpair(e.k, q) == e.b) {
                    wblk[(e.k * 2 + p) * 2 + q] += e.coef;
                    placed = true;
                }
        if (!placed) throw std::runtime_error("RT0 mass entry does not match the star edge pairs");
    }
    std::vector<DevPatchClass<double>> c64 = convert_classes<double>(cls);
    // the variable-K smoother solves interior-tile patches with every slot taken as present
    for (int a = 0; a < PATCH; ++a)
        if (!c64[4].present[a]) throw std::runtime_error("interior patch class with an absent slot");
    upload(lv.cls64, c64, st);
    upload(lv.wblk64, wblk, st);
    std::vector<DevPatchClass<float>> c32 = convert_classes<float>(cls);
    std::vector<float> wblk32(wblk.begin(), wblk.end());
    upload(lv.cls32, c32, st);
    upload(lv.wblk32, wblk32, st);
    if (uniform) {
        // inverse of each class's patch matrix, column by column (zero rows and columns on
        // absent DoFs; zero for the pressure-only corner classes)
        std::vector<double> minv(9 * PATCH * PATCH, 0.0);
        const double kv[6] = {Kinv, Kinv, Kinv, Kinv, Kinv, Kinv};
        for (int k = 0; k < 9; ++k)
            for (int j = 0; j < PATCH; ++j) {
                if (!c64[k].present[j]) continue;
                double e[PATCH] = {0}, col[PATCH];
                e[j] = 1.0;
                patch_solve<double>(e, c64[k], kv, wblk.data(), col, 1);
                for (int a = 0; a < PATCH; ++a) minv[(k * PATCH + a) * PATCH + j] = c64[k].present[a] ? col[a] : 0.0;
            }
        upload(lv.minv64, minv, st);
    } else {
        lv.minv64.release();
    }
    UPatchClass ucls[9];
    build_upatch_classes(lv.st_host, lv.n, ucls);
    upload(lv.uinv64, convert_uinv<double>(ucls), st);
    upload(lv.uinv32, convert_uinv<float>(ucls), st);
}

// reject a per-triangle field (2 n^2 device values) with an unusable value before anything
// changes: mode 0 permeabilities, mode 1 log-permeabilities (synchronizes the stream)
static void check_field(biot_ctx* c, const double* v, int mode, hipStream_t st) {
    launch_check_field(v, 2LL * c->n * c->n, mode, c->kcheck.as<int>(), st);
    check_stream_error();
    int bad = 0;
    BIOT_HIP(hipMemcpyAsync(&bad, c->kcheck.p, sizeof(int), hipMemcpyDeviceToHost, st));
    BIOT_HIP(hipStreamSynchronize(st));
    if (bad)
        throw ArgError{mode == 0 ? "permeability: every K must be finite and > 0 with 1/K finite"
                                 : "log-permeability: every theta = ln K must be finite with |theta| < 700"};
}

// 1/K on every level from the finest level's (mode 0: K_tri, or K_scalar if null; mode 1:
// exp(-theta))
static void levels_kinv(biot_ctx* c, const double* K_tri, hipStream_t st, int mode = 0) {
    Level& l0 = *c->levels[0];
    if (mode == 0)
        launch_kinv_from_K(K_tri, c->K_scalar, l0.kinv64.as<double>(), l0.L, st);
    else
        launch_kinv_from_logK(K_tri, l0.kinv64.as<double>(), l0.L, st);
    for (size_t l = 1; l < c->levels.size(); ++l)
        launch_kinv_coarsen(c->levels[l - 1]->kinv64.as<double>(), c->levels[l - 1]->L,
                            c->levels[l]->kinv64.as<double>(), c->levels[l]->L, st);
    for (auto& lv : c->levels) launch_convert(lv->kinv64.as<double>(), lv->kinv32.as<float>(), 2 * lv->L.plane, st);
}

// Variable K: the factors of every vertex patch of the smoothing levels with at most FAC_MAX_N
// cells per side, from the current 1/K (they depend on the permeability only; a relaxation step
// applies them).  Measured on the 2048 x 2048 block-contrast hierarchy: stored factors shorten
// a colour step at 512^2 (52 us against 60 us) and lengthen it at 1024^2 and 2048^2 (208 against
// 201 us, 829 against 768 us), where their loads (336 B per patch, read through partial cache
// lines in a colour step) cost more than forming them on the spot.
constexpr int FAC_MAX_N = 512;
static void levels_factors(biot_ctx* c, hipStream_t st) {
    if (c->K_uniform) return;
    for (size_t l = 0; l + 1 < c->levels.size(); ++l) {
        Level& lv = *c->levels[l];
        if (lv.n > FAC_MAX_N) continue;
        if (!lv.fac64.p) lv.fac64.alloc((size_t)PFAC * lv.L.plane * sizeof(double));
        launch_patch_factors(lv.view<double>(), lv.fac64.as<double>(), st);
    }
}

// BSR diagonal data of every smoothing level from the current 1/K (Appendix D)
static void levels_bsr(biot_ctx* c, hipStream_t st) {
    const PhysParams& p = c->phys;
    const double cu = p.inv_M + p.alpha * p.alpha / (p.lambda + p.mu);
    for (size_t l = 0; l + 1 < c->levels.size(); ++l) {
        Level& lv = *c->levels[l];
        const size_t len = (size_t)lv.L.len;
        if (!lv.bsrd64.p) {
            lv.bsrd64.alloc(5 * lv.L.plane * sizeof(double));
            lv.bsrd32.alloc(5 * lv.L.plane * sizeof(float));
            // the diagonal kernels write the mesh slots only; the ghost ring stays zero
            launch_fill(lv.bsrd64.as<double>(), 5 * lv.L.plane, 0.0, st);
            launch_fill(lv.bsrd32.as<float>(), 5 * lv.L.plane, 0.0f, st);
            lv.bs64.alloc(len * sizeof(double));
            lv.bs32.alloc(len * sizeof(float));
            launch_fill(lv.bs64.as<double>(), lv.L.len, 0.0, st);
            launch_fill(lv.bs32.as<float>(), lv.L.len, 0.0f, st);
            lv.sch64.alloc(10 * lv.L.plane * sizeof(double));
            lv.sch32.alloc(10 * lv.L.plane * sizeof(float));
            launch_fill(lv.sch64.as<double>(), 10 * lv.L.plane, 0.0, st);
            launch_fill(lv.sch32.as<float>(), 10 * lv.L.plane, 0.0f, st);
            lv.cgred.alloc((2 * (size_t)cg_partials(lv.L) + 3) * sizeof(double));
            launch_fill(lv.cgred.as<double>(), 2LL * cg_partials(lv.L) + 3, 0.0, st);
        }
        const double area = 0.5 * lv.h * lv.h;
        lv.cS = cu * area;
        launch_bsr_diag<double>(lv.view<double>(), cu * area, lv.bsrd64.as<double>(), st);
        launch_convert(lv.bsrd64.as<double>(), lv.bsrd32.as<float>(), 5 * lv.L.plane, st);
    }
}

static void coarse_setup(biot_ctx* c, hipStream_t st) {
    Level& lc = *c->levels.back();
    const Layout& L = lc.L;
    std::vector<int> idx, map((size_t)L.len, -1);
    for (int t = 0; t < NTYPES; ++t)
        for (int j = 0; j <= L.n; ++j)
            for (int i = 0; i <= L.n; ++i)
                if (dof_free(t, i, j, L.n)) {
                    long long p = t * L.plane + slot_index(L, i, j);
                    map[(size_t)p] = (int)idx.size();
                    idx.push_back((int)p);
                }
    const int N = (int)idx.size();
    c->coarse_N = N;
    upload(c->coarse_idx, idx, st);
    upload(c->coarse_map, map, st);
    c->coarse_A.alloc((size_t)N * N * sizeof(double));
    c->coarse_inv.alloc((size_t)N * N * sizeof(double));
    c->coarse_col.alloc((size_t)N * sizeof(double));
    c->status.alloc(sizeof(int));
}

static void coarse_factor(biot_ctx* c, hipStream_t st) {
    Level& lc = *c->levels.back();
    const int N = c->coarse_N;
    launch_coarse_matrix(lc.L, lc.st.as<StencilEntry>(), lc.st_off.as<int>(), lc.kinv64.as<double>(),
                         c->coarse_idx.as<int>(), c->coarse_map.as<int>(), N, c->coarse_A.as<double>(), st);
    launch_gauss_jordan(c->coarse_A.as<double>(), c->coarse_inv.as<double>(), N, c->coarse_col.as<double>(),
                        c->status.as<int>(), st);
    check_stream_error();
    int status = 0;
    BIOT_HIP(hipMemcpyAsync(&status, c->status.p, sizeof(int), hipMemcpyDeviceToHost, st));
    BIOT_HIP(hipStreamSynchronize(st));
    if (status != 0) throw SingularError{"coarsest-level operator is singular"};
}

// ---- V-cycle -----------------------------------------------------------------------------------------
template <typename T>
struct VecSet;
template <>
struct VecSet<double> {
    static double* x(Level& l) { return l.x64.as<double>(); }
    static double* b(Level& l) { return l.b64.as<double>(); }
    static double* r(Level& l) { return l.r64.as<double>(); }
    static double* s(Level& l) { return l.bs64.as<double>(); }
    static double* sch(Level& l) { return l.sch64.as<double>(); }
};
template <>
struct VecSet<float> {
    static float* x(Level& l) { return l.x32.as<float>(); }
    static float* b(Level& l) { return l.b32.as<float>(); }
    static float* r(Level& l) { return l.r32.as<float>(); }
    static float* s(Level& l) { return l.bs32.as<float>(); }
    static float* sch(Level& l) { return l.sch32.as<float>(); }
};

// Event pair for one launch when kernel timing is on for this level (kind 0 Vanka, 1 residual):
// the launch records the kernel's own start and end in it.  Null events otherwise.
static LaunchTiming prof_events(biot_ctx* c, int kind, int level) {
    LaunchTiming t;
    if (!c->prof_on || level != c->prof_level) return t;
    auto& pool = c->prof_ev[kind];
    size_t& used = c->prof_used[kind];
    while (pool.size() < used + 2) {
        hipEvent_t e;
        BIOT_HIP(hipEventCreate(&e));
        pool.push_back(e);
    }
    t.start = pool[used];
    t.stop = pool[used + 1];
    used += 2;
    return t;
}

// The two iterate buffers of a level (the fused Vanka step reads one and writes the other).
template <typename T>
struct XBuf;
template <>
struct XBuf<double> {
    static double* get(Level& l, int k) { return (k ? l.x2_64 : l.x64).as<double>(); }
};
template <>
struct XBuf<float> {
    static float* get(Level& l, int k) { return (k ? l.x2_32 : l.x32).as<float>(); }
};

// BSR Schur sweeps of level l (sweeps <= 1: the single step, no descriptor needed)
template <typename T>
static SchurSweeps<T> schur_sweeps(biot_ctx* c, Level& lv) {
    SchurSweeps<T> sw{c->opts.schur_sweeps, (T)c->opts.omega_S, (T)lv.cS, VecSet<T>::sch(lv)};
    sw.cg = c->opts.schur_cg;
    sw.red = lv.cgred.as<double>();
    return sw;
}

// Multiplicative Vanka: the colours of a step are separate launches, each reading the iterate
// the previous one wrote.
static int vanka_colors(const biot_mg_opts& o) {
    return o.smoother == BIOT_SMOOTHER_VANKA && (o.vanka_colors == 3 || o.vanka_colors == 4) ? o.vanka_colors : 1;
}

// colours and weight of level l: the finest additive_levels levels take the additive step
static int vanka_colors_at(const biot_mg_opts& o, int l) { return l < o.additive_levels ? 1 : vanka_colors(o); }
static double omega_at(const biot_mg_opts& o, int l) {
    return l < o.additive_levels && o.omega_additive > 0 ? o.omega_additive : o.omega;
}

// the kernel's colour code of colour col of nc (-1: the additive step)
static int color_code(int nc, int col) { return nc == 4 ? col : (nc == 3 ? 4 + col : -1); }

// One relaxation step on level l from the iterate x (nullptr: zero).  Vanka writes the new
// iterate to dst (dst != x); its multiplicative form alternates between dst and alt (the other
// buffer of the pair, != dst) and returns the buffer it ended in.  BSR updates in place
// (dst == x, or x == nullptr).  Returns the buffer holding the new iterate.
template <typename T>
static T* relax(biot_ctx* c, int l, const T* x, const T* b, T* dst, T* alt, hipStream_t st) {
    Level& lv = *c->levels[l];
    LevelView<T> v = lv.view<T>();
    const T om = (T)omega_at(c->opts, l);
    if (c->opts.smoother == BIOT_SMOOTHER_VANKA) {
        const int nc = vanka_colors_at(c->opts, l);
        if (nc > 1 && (!alt || alt == dst)) throw ArgError{"multiplicative Vanka needs a second buffer"};
        const T* src = x;
        T* out = dst;
        for (int col = 0; col < nc; ++col) {
            const LaunchTiming tm = src ? prof_events(c, 0, l) : LaunchTiming{};
            launch_vanka_step<T>(v, src, b, out, c->K_uniform, (T)(1.0 / c->K_scalar), om, st, nullptr, nullptr,
                                 nullptr, &tm, color_code(nc, col));
            src = out;
            out = out == dst ? alt : dst;
        }
        return const_cast<T*>(src);
    }
    const SchurSweeps<T> sw = schur_sweeps<T>(c, lv);
    launch_bsr_step<T>(v, dst, b, VecSet<T>::r(lv), VecSet<T>::s(lv), x == nullptr, c->K_uniform,
                       (T)(1.0 / c->K_scalar), om, (T)c->opts.omega_J, nullptr, nullptr, nullptr, nullptr, st, &sw);
    return dst;
}

// Times the iterate moves to the other buffer during the smoothing on one level (the first
// step from zero writes buffer 0).
static int buffer_moves(const biot_mg_opts& o, int l) {
    if (o.smoother != BIOT_SMOOTHER_VANKA) return 0;
    const int nc = vanka_colors_at(o, l);
    return (o.nu1 > 0 ? o.nu1 * nc - 1 : 0) + o.nu2 * nc;
}

template <typename T>
struct PW;
template <>
struct PW<double> {
    static const double* get(biot_ctx* c) { return c->pw64.as<double>(); }
};
template <>
struct PW<float> {
    static const float* get(biot_ctx* c) { return c->pw32.as<float>(); }
};

static double* small_entry(biot_ctx* c, const double* b, double* buf0, double* x0, bool vonly, hipStream_t st);

// V(nu1, nu2) cycle on level l for A_l x = b from x = 0 (or from x0), iterate buffers buf0 / buf1
// (both zero on absent DoFs).  Returns the buffer that holds the result.  vonly: no level below
// repeats its coarse correction (the V-cycles of an F-cycle).
template <typename T>
static T* vcycle_level(biot_ctx* c, int l, const T* b, T* buf0, T* buf1, hipStream_t st, T* x0 = nullptr,
                       bool vonly = false) {
    Level& lv = *c->levels[l];
    if (c->small && l == c->small_from) {
        // the small levels run on CSR operators and explicit patch inverses, in FP64
        if constexpr (std::is_same_v<T, double>) {
            return small_entry(c, b, buf0, x0, vonly, st);
        } else {
            // FP32 forms: through the level's FP64 buffers (zero on absent DoFs)
            double* bd = lv.b64.as<double>();
            double* xd = lv.x64.as<double>();
            launch_convert(b, bd, lv.L.len, st);
            if (x0) launch_convert(x0, xd, lv.L.len, st);
            double* r = small_entry(c, bd, lv.x2_64.as<double>(), x0 ? xd : nullptr, vonly, st);
            launch_convert(r, buf0, lv.L.len, st);
            return buf0;
        }
    }
    if (l == (int)c->levels.size() - 1) {
        launch_coarse_solve<T>(c->coarse_inv.as<double>(), c->coarse_N, c->coarse_idx.as<int>(), b, buf0, st);
        return buf0;
    }
    const bool inplace = c->opts.smoother != BIOT_SMOOTHER_VANKA;
    // the iterate: zero, or x0 (buf0 or buf1) when the cycle continues from a previous one
    T* cur = x0;
    auto next = [&]() { return cur == nullptr ? buf0 : (inplace ? cur : (cur == buf0 ? buf1 : buf0)); };
    auto other = [&](T* d) { return d == buf0 ? buf1 : buf0; };
    for (int s = 0; s < c->opts.nu1; ++s) {
        T* d = next();
        cur = relax<T>(c, l, cur, b, d, other(d), st);
    }
    if (!cur) {
        launch_fill(buf0, lv.L.len, (T)0, st);
        cur = buf0;
    }
    Level& lc = *c->levels[l + 1];
    T* bc = VecSet<T>::b(lc);
    const LaunchTiming tm = prof_events(c, 1, l);
    launch_residual_restrict<T>(lv.view<T>(), lc.L, cur, b, bc, c->K_uniform, (T)(1.0 / c->K_scalar),
                                PW<T>::get(c), st, &tm);
    T* xc = vcycle_level<T>(c, l + 1, bc, XBuf<T>::get(lc, 0), XBuf<T>::get(lc, 1), st, nullptr, vonly);
    if (!vonly && c->opts.gamma > 1 && l >= c->opts.gamma_from && (c->opts.gamma_to == 0 || l < c->opts.gamma_to) &&
        l + 2 < (int)c->levels.size()) {
        // W-cycle: gamma - 1 further cycles of level l + 1, each continuing from the iterate the
        // previous one left (with linear smoothing the same as a cycle from zero on the residual
        // it left, added to it); the coarsest level's direct solve is exact and not repeated.
        // F-cycle: the further cycles are V-cycles.
        for (int g = 1; g < c->opts.gamma; ++g)
            xc = vcycle_level<T>(c, l + 1, bc, XBuf<T>::get(lc, 0), XBuf<T>::get(lc, 1), st, xc,
                                 c->opts.fcycle != 0);
    }
    int s0 = 0;
    if (c->opts.nu2 > 0) {
        // prolongation fused into the first post-smoothing step
        const T kinv_s = (T)(1.0 / c->K_scalar);
        if (!inplace) {
            // multiplicative form: colour 0 with the prolongation, then colours 1..3
            const int nc = vanka_colors_at(c->opts, l);
            for (int col = 0; col < nc; ++col) {
                T* dst = next();
                launch_vanka_step<T>(lv.view<T>(), cur, b, dst, c->K_uniform, kinv_s, (T)omega_at(c->opts, l), st,
                                     col == 0 ? xc : nullptr, &lc.L, PW<T>::get(c), nullptr, color_code(nc, col));
                cur = dst;
            }
        } else {
            T* other = cur == buf0 ? buf1 : buf0;
            const SchurSweeps<T> sw = schur_sweeps<T>(c, lv);
            launch_bsr_step<T>(lv.view<T>(), cur, b, VecSet<T>::r(lv), VecSet<T>::s(lv), false, c->K_uniform, kinv_s,
                               (T)c->opts.omega, (T)c->opts.omega_J, xc, &lc.L, PW<T>::get(c), other, st, &sw);
        }
        s0 = 1;
    } else {
        launch_prolong_add<T>(lv.L, lc.L, xc, cur, PW<T>::get(c), st);
    }
    for (int s = s0; s < c->opts.nu2; ++s) {
        T* d = next();
        cur = relax<T>(c, l, cur, b, d, other(d), st);
    }
    return cur;
}

// ---- general-boundary path (sparse.h) -----------------------------------------------------------
// Level l of the path: numbering, CSR pattern and assembly lists, per-triangle 1/K and work vectors.
static void sp_level_alloc(SpLevel& L, int n, int bc, const PhysParams& p, hipStream_t st) {
    L.map = make_free_map(n, bc);
    OperatorHost op = build_operator(L.map, p);
    L.N = L.map.N;
    L.nnz = (int)op.A.col.size();
    L.ptr_h = op.A.ptr;
    upload(L.ptr, op.A.ptr, st);
    upload(L.col, op.A.col, st);
    upload(L.val0, op.A.val, st);
    upload(L.kptr, op.kptr, st);
    upload(L.ktri, op.ktri, st);
    upload(L.kcoef, op.kcoef, st);
    L.val.alloc((size_t)std::max(1, L.nnz) * sizeof(double));
    L.kinv.alloc((size_t)2 * n * n * sizeof(double));
    for (DevBuf* b : {&L.x, &L.b, &L.r}) {
        b->alloc((size_t)L.N * sizeof(double));
        launch_fill(b->as<double>(), L.N, 0.0, st);
    }
    BIOT_HIP(hipStreamSynchronize(st));   // the host tables above go out of scope
}

// transfers between level l (fine) and l + 1, and the Vanka patches of level l
static void sp_level_links(SpLevel& F, const SpLevel& C, hipStream_t st, int ncolors = 1,
                           const std::vector<int>* rowptr = nullptr) {
    const CsrHost P = build_prolongation(F.map, C.map);
    const CsrHost R = csr_transpose(P);
    upload(F.pptr, P.ptr, st);
    upload(F.pcol, P.col, st);
    upload(F.pval, P.val, st);
    upload(F.rptr, R.ptr, st);
    upload(F.rcol, R.col, st);
    upload(F.rval, R.val, st);
    std::vector<int> verts;
    const std::vector<int> slots = build_patches(F.map, &verts);
    F.np = (int)(slots.size() / PATCH);
    if (ncolors > 1) {
        // the colours of the structured kernels: (i mod 2) + 2 (j mod 2), or (i + 2 j) mod 3
        std::vector<int> clist;
        F.coff.assign((size_t)ncolors + 1, 0);
        const int n1 = F.map.n + 1;
        for (int col = 0; col < ncolors; ++col) {
            for (int p = 0; p < F.np; ++p) {
                const int i = verts[p] % n1, j = verts[p] / n1;
                const int cp = ncolors == 4 ? (i & 1) + 2 * (j & 1) : (i + 2 * j) % 3;
                if (cp == col) clist.push_back(p);
            }
            F.coff[(size_t)col + 1] = (int)clist.size();
        }
        upload(F.clist, clist, st);
        if (rowptr) {
            std::vector<int> crow(clist.size() * PATCH), cbeg(crow.size(), 0), cend(crow.size(), 0);
            for (size_t k = 0; k < clist.size(); ++k)
                for (int a = 0; a < PATCH; ++a) {
                    const int d = slots[(size_t)clist[k] * PATCH + a];
                    const size_t e = k * PATCH + a;
                    crow[e] = d;
                    if (d >= 0) {
                        cbeg[e] = (*rowptr)[(size_t)d];
                        cend[e] = (*rowptr)[(size_t)d + 1];
                    }
                }
            upload(F.crow, crow, st);
            upload(F.cbeg, cbeg, st);
            upload(F.cend, cend, st);
            // a zero-start colour 0 also writes the zeros of the DoFs its patches do not hold
            std::vector<char> cov((size_t)F.N, 0);
            for (size_t e = 0; e < (size_t)F.coff[1] * PATCH; ++e)
                if (crow[e] >= 0) cov[(size_t)crow[e]] = 1;
            std::vector<int> zl;
            for (int d = 0; d < F.N; ++d)
                if (!cov[(size_t)d]) zl.push_back(d);
            F.nz0 = (int)zl.size();
            upload(F.zlist0, zl, st);
        }
    }
    // DoF -> (patch, slot) lists in patch order (a fixed summation order) and D = 1 / count
    std::vector<int> dptr((size_t)F.N + 1, 0), dlist;
    for (int q : slots)
        if (q >= 0) ++dptr[(size_t)q + 1];
    for (int d = 0; d < F.N; ++d) dptr[(size_t)d + 1] += dptr[d];
    dlist.resize((size_t)dptr[F.N]);
    std::vector<int> fill(dptr.begin(), dptr.end() - 1);
    for (size_t e = 0; e < slots.size(); ++e)
        if (slots[e] >= 0) dlist[(size_t)fill[slots[e]]++] = (int)e;
    std::vector<double> wgt((size_t)F.N);
    for (int d = 0; d < F.N; ++d) {
        const int cnt = dptr[(size_t)d + 1] - dptr[d];
        if (cnt == 0) throw std::runtime_error("a free DoF lies in no Vanka patch");
        wgt[d] = 1.0 / cnt;
    }
    upload(F.slots, slots, st);
    upload(F.dptr, dptr, st);
    upload(F.dlist, dlist, st);
    upload(F.wgt, wgt, st);
    F.inv.alloc((size_t)std::max(1, F.np) * PATCH * PATCH * sizeof(double));
    F.y.alloc((size_t)std::max(1, F.np) * PATCH * sizeof(double));
    BIOT_HIP(hipStreamSynchronize(st));   // the host tables above go out of scope
}

// 1/K of every level from the finest level's field (mode 0: K_tri, or the scalar when null;
// mode 1: theta = ln K), then the operator values of every level
static void sp_assemble(biot_ctx* c, const double* field, int mode, hipStream_t st) {
    SpHier& H = *c->sp;
    launch_kinv_flat(2LL * c->n * c->n, field, c->K_scalar, mode, H.lv[0]->kinv.as<double>(), st);
    for (size_t l = 1; l < H.lv.size(); ++l)
        launch_kinv_coarsen_flat(c->n >> l, H.lv[l - 1]->kinv.as<double>(), H.lv[l]->kinv.as<double>(), st);
    for (auto& lp : H.lv)
        launch_csr_assemble(lp->nnz, lp->val0.as<double>(), lp->kptr.as<int>(), lp->ktri.as<int>(),
                            lp->kcoef.as<double>(), lp->kinv.as<double>(), lp->val.as<double>(), st);
}

// the permeability-dependent set-up of the hierarchy: patch inverses and the coarsest inverse
static void sp_factor(biot_ctx* c, hipStream_t st) {
    SpHier& H = *c->sp;
    int* status = H.status.as<int>();
    BIOT_HIP(hipMemsetAsync(status, 0, sizeof(int), st));
    for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
        SpLevel& L = *H.lv[l];
        launch_patch_inverse(L.np, L.slots.as<int>(), L.ptr.as<int>(), L.col.as<int>(), L.val.as<double>(),
                             c->opts.vanka_shift, L.inv.as<double>(), status, st);
    }
    check_stream_error();
    int bad = 0;
    BIOT_HIP(hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, st));
    BIOT_HIP(hipStreamSynchronize(st));
    if (bad) throw SingularError{"a Vanka patch matrix is singular (with 1/M = 0 set vanka_shift > 0)"};
    SpLevel& C = *H.lv.back();
    launch_csr_to_dense(H.cN, C.ptr.as<int>(), C.col.as<int>(), C.val.as<double>(), H.cA.as<double>(), st);
    launch_gauss_jordan(H.cA.as<double>(), H.cinv.as<double>(), H.cN, H.ccol.as<double>(), status, st);
    check_stream_error();
    BIOT_HIP(hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, st));
    BIOT_HIP(hipStreamSynchronize(st));
    if (bad) throw SingularError{"coarsest-level operator is singular"};
}

static void sp_setup(biot_ctx* c, const biot_mg_opts* o, hipStream_t st) {
    SpHier& H = *c->sp;
    c->have_hierarchy = false;
    H.lv.resize(1);
    for (int l = 1; l < o->levels; ++l) {
        H.lv.emplace_back(new SpLevel);
        sp_level_alloc(*H.lv[l], c->n >> l, H.bc, c->phys, st);
    }
    for (int l = 0; l + 1 < o->levels; ++l) sp_level_links(*H.lv[l], *H.lv[l + 1], st);
    H.cN = H.lv.back()->N;
    H.cA.alloc((size_t)H.cN * H.cN * sizeof(double));
    H.cinv.alloc((size_t)H.cN * H.cN * sizeof(double));
    H.ccol.alloc((size_t)H.cN * sizeof(double));
    std::vector<int> idx((size_t)H.cN);
    for (int k = 0; k < H.cN; ++k) idx[k] = k;
    upload(H.cidx, idx, st);
    H.status.alloc(sizeof(int));
    c->opts = *o;
    if (c->opts.gamma < 1) c->opts.gamma = 1;
    // coarse 1/K from the finest level's (still in lv[0].kinv), then every operator
    for (size_t l = 1; l < H.lv.size(); ++l)
        launch_kinv_coarsen_flat(c->n >> l, H.lv[l - 1]->kinv.as<double>(), H.lv[l]->kinv.as<double>(), st);
    for (size_t l = 1; l < H.lv.size(); ++l) {
        SpLevel& L = *H.lv[l];
        launch_csr_assemble(L.nnz, L.val0.as<double>(), L.kptr.as<int>(), L.ktri.as<int>(), L.kcoef.as<double>(),
                            L.kinv.as<double>(), L.val.as<double>(), st);
    }
    sp_factor(c, st);
    c->have_hierarchy = true;
}

// y = A_l x (mode 0) or y = b - A_l x (mode 1) on compact vectors of level l
static void sp_apply(biot_ctx* c, int l, const double* x, const double* b, double* y, int mode, hipStream_t st) {
    SpLevel& L = *c->sp->lv[l];
    launch_csr_mv(L.N, L.ptr.as<int>(), L.col.as<int>(), L.val.as<double>(), x, mode == 1 ? b : nullptr, y,
                  mode == 1 ? -1.0 : 1.0, 1.0, st);
}

// one additive Vanka step x <- x + omega sum_l V_l^T D_l A_l^{-1} V_l (b - A x) in place
// (zero: x = 0 on entry, the residual is b)
static void sp_smooth_level(SpLevel& L, double omega, double* x, const double* b, bool zero, hipStream_t st) {
    const double* r = b;
    if (!zero) {
        launch_csr_mv(L.N, L.ptr.as<int>(), L.col.as<int>(), L.val.as<double>(), x, b, L.r.as<double>(), -1.0, 1.0,
                      st);
        r = L.r.as<double>();
    }
    launch_patch_apply(L.np, L.slots.as<int>(), L.inv.as<double>(), r, L.y.as<double>(), st);
    launch_patch_gather(L.N, L.dptr.as<int>(), L.dlist.as<int>(), L.y.as<double>(), L.wgt.as<double>(), omega,
                        zero ? nullptr : x, x, st);
}

static void sp_smooth(biot_ctx* c, int l, double* x, const double* b, bool zero, hipStream_t st) {
    sp_smooth_level(*c->sp->lv[l], c->opts.omega, x, b, zero, st);
}

// The cycle on level l for A_l x = b, from x = 0 (zero) or from the iterate in x, result in x
// (b != x).  The coarse problem lives in the next level's b and x; a repeated coarse visit
// continues from the coarse iterate (the same as a cycle on the remaining residual, added).
static void sp_cycle(biot_ctx* c, int l, const double* b, double* x, bool zero, bool vonly, hipStream_t st) {
    SpHier& H = *c->sp;
    const int nl = (int)H.lv.size();
    if (l == nl - 1) {
        launch_coarse_solve<double>(H.cinv.as<double>(), H.cN, H.cidx.as<int>(), b, x, st);
        return;
    }
    const biot_mg_opts& o = c->opts;
    SpLevel& L = *H.lv[l];
    SpLevel& C = *H.lv[l + 1];
    bool z = zero;
    for (int s = 0; s < o.nu1; ++s, z = false) sp_smooth(c, l, x, b, z, st);
    if (z) launch_fill(x, L.N, 0.0, st);
    sp_apply(c, l, x, b, L.r.as<double>(), 1, st);
    launch_csr_mv(C.N, L.rptr.as<int>(), L.rcol.as<int>(), L.rval.as<double>(), L.r.as<double>(), nullptr,
                  C.b.as<double>(), 1.0, 0.0, st);
    sp_cycle(c, l + 1, C.b.as<double>(), C.x.as<double>(), true, vonly, st);
    const bool repeat = !vonly && l + 1 < nl - 1 && l >= o.gamma_from && (o.gamma_to <= 0 || l < o.gamma_to);
    if (repeat)
        for (int g = 1; g < o.gamma; ++g) sp_cycle(c, l + 1, C.b.as<double>(), C.x.as<double>(), false, o.fcycle != 0, st);
    launch_csr_mv(L.N, L.pptr.as<int>(), L.pcol.as<int>(), L.pval.as<double>(), C.x.as<double>(), x, x, 1.0, 1.0, st);
    for (int s = 0; s < o.nu2; ++s) sp_smooth(c, l, x, b, false, st);
}

// ---- small levels of the Dirichlet path on CSR (opts.csr_below) ---------------------------------
// Below some size a level's fused stencil launch is bound by the latency chain of one block
// (about 15 us whatever the level's size), while the CSR residual and the explicit-inverse patch
// apply take a few microseconds each.  Levels small_from .. L-2 then smooth on CSR operators
// (the same rediscretization, assembled from the same per-triangle 1/K) with explicit patch
// inverses; the coarsest level keeps its dense inverse (in the canonical order, which is the
// compact order of these levels).  Their vectors are compact; the finer structured level hands
// its restricted residual over by an unpack and takes the result back by a pack.

// 1/K, operator values and patch inverses of the small levels from the structured levels' 1/K
static void small_refresh(biot_ctx* c, hipStream_t st) {
    SpHier& H = *c->small;
    int* status = H.status.as<int>();
    BIOT_HIP(hipMemsetAsync(status, 0, sizeof(int), st));
    for (size_t k = 0; k < H.lv.size(); ++k) {
        SpLevel& L = *H.lv[k];
        const Level& lv = *c->levels[(size_t)c->small_from + k];
        launch_kinv_unpad(lv.L, lv.kinv64.as<double>(), L.kinv.as<double>(), st);
        launch_csr_assemble(L.nnz, L.val0.as<double>(), L.kptr.as<int>(), L.ktri.as<int>(), L.kcoef.as<double>(),
                            L.kinv.as<double>(), L.val.as<double>(), st);
        if (k + 1 < H.lv.size())
            launch_patch_inverse(L.np, L.slots.as<int>(), L.ptr.as<int>(), L.col.as<int>(), L.val.as<double>(), 0.0,
                                 L.inv.as<double>(), status, st);
    }
    check_stream_error();
    int bad = 0;
    BIOT_HIP(hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, st));
    BIOT_HIP(hipStreamSynchronize(st));
    if (bad) throw SingularError{"a Vanka patch matrix of a small level is singular"};
}

static void small_setup(biot_ctx* c, hipStream_t st) {
    c->small.reset();
    c->small_from = -1;
    const biot_mg_opts& o = c->opts;
    if (o.csr_below <= 0) return;
    const int L = (int)c->levels.size();
    int s = 1;
    while (s < L - 1 && (c->n >> s) > o.csr_below) ++s;
    if (s >= L - 1) return;                      // no smoothing level is that small
    std::unique_ptr<SpHier> H(new SpHier);
    H->bc = BC_DIRICHLET;
    for (int l = s; l < L; ++l) {
        H->lv.emplace_back(new SpLevel);
        sp_level_alloc(*H->lv.back(), c->n >> l, BC_DIRICHLET, c->phys, st);
    }
    for (size_t k = 0; k + 1 < H->lv.size(); ++k)
        sp_level_links(*H->lv[k], *H->lv[k + 1], st, vanka_colors_at(o, s + (int)k), &H->lv[k]->ptr_h);
    std::vector<int> idx((size_t)c->coarse_N);
    for (int k = 0; k < c->coarse_N; ++k) idx[k] = k;
    upload(H->cidx, idx, st);
    H->status.alloc(sizeof(int));
    c->small = std::move(H);
    c->small_from = s;
    small_refresh(c, st);
}

// one smoothing step on small level g (additive, or the colours in turn), x in place
static void small_smooth(biot_ctx* c, int g, SpLevel& L, double* x, const double* b, bool zero, hipStream_t st) {
    const int nc = vanka_colors_at(c->opts, g);
    const double om = omega_at(c->opts, g);
    if (nc == 1) {
        sp_smooth_level(L, om, x, b, zero, st);
        return;
    }
    for (int col = 0; col < nc; ++col) {
        const size_t o = (size_t)L.coff[col] * PATCH;
        launch_colour_step(L.coff[(size_t)col + 1] - L.coff[col], L.clist.as<int>() + L.coff[col],
                           L.crow.as<int>() + o, L.cbeg.as<int>() + o, L.cend.as<int>() + o, L.inv.as<double>(),
                           L.col.as<int>(), L.val.as<double>(), b, x, om, zero && col == 0, st, L.zlist0.as<int>(),
                           L.nz0);
    }
}

// the cycle on small level k (global level small_from + k), as vcycle_level: from zero or from
// the iterate in x, result in x; the same repetition rule
static void small_cycle(biot_ctx* c, int k, const double* b, double* x, bool zero, bool vonly, hipStream_t st) {
    SpHier& H = *c->small;
    const int g = c->small_from + k;
    const int nl = (int)c->levels.size();
    if (g == nl - 1) {
        launch_coarse_solve<double>(c->coarse_inv.as<double>(), c->coarse_N, H.cidx.as<int>(), b, x, st);
        return;
    }
    const biot_mg_opts& o = c->opts;
    SpLevel& L = *H.lv[k];
    SpLevel& C = *H.lv[(size_t)k + 1];
    bool z = zero;
    for (int s = 0; s < o.nu1; ++s, z = false) small_smooth(c, g, L, x, b, z, st);
    if (z) launch_fill(x, L.N, 0.0, st);
    launch_csr_mv(L.N, L.ptr.as<int>(), L.col.as<int>(), L.val.as<double>(), x, b, L.r.as<double>(), -1.0, 1.0, st);
    launch_csr_mv(C.N, L.rptr.as<int>(), L.rcol.as<int>(), L.rval.as<double>(), L.r.as<double>(), nullptr,
                  C.b.as<double>(), 1.0, 0.0, st);
    small_cycle(c, k + 1, C.b.as<double>(), C.x.as<double>(), true, vonly, st);
    if (!vonly && o.gamma > 1 && g >= o.gamma_from && (o.gamma_to == 0 || g < o.gamma_to) && g + 2 < nl)
        for (int gg = 1; gg < o.gamma; ++gg)
            small_cycle(c, k + 1, C.b.as<double>(), C.x.as<double>(), false, o.fcycle != 0, st);
    launch_csr_mv(L.N, L.pptr.as<int>(), L.pcol.as<int>(), L.pval.as<double>(), C.x.as<double>(), x, x, 1.0, 1.0, st);
    for (int s = 0; s < o.nu2; ++s) small_smooth(c, g, L, x, b, false, st);
}

// entry from the structured cycle at level small_from: b and x0 (or nullptr) padded; the result
// is packed into buf0 (zero on absent DoFs, as every iterate buffer)
static double* small_entry(biot_ctx* c, const double* b, double* buf0, double* x0, bool vonly, hipStream_t st) {
    const Level& lv = *c->levels[c->small_from];
    SpLevel& L = *c->small->lv[0];
    launch_unpack(b, L.b.as<double>(), lv.L, lv.C, st);
    if (x0) launch_unpack(x0, L.x.as<double>(), lv.L, lv.C, st);
    small_cycle(c, 0, L.b.as<double>(), L.x.as<double>(), x0 == nullptr, vonly, st);
    launch_pack(L.x.as<double>(), buf0, lv.L, lv.C, st);
    return buf0;
}

// vector length of the Krylov solve: padded finest level, or the compact free DoFs
static long long vec_len(biot_ctx* c) { return c->sp ? (long long)c->sp->lv[0]->N : c->levels[0]->L.len; }

static void vec_pack(biot_ctx* c, const double* canon, double* v, hipStream_t st) {
    if (c->sp) {
        BIOT_HIP(hipMemcpyAsync(v, canon, (size_t)vec_len(c) * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
        Level& l0 = *c->levels[0];
        launch_pack(canon, v, l0.L, l0.C, st);
    }
}

static void vec_unpack(biot_ctx* c, const double* v, double* canon, hipStream_t st) {
    if (c->sp) {
        BIOT_HIP(hipMemcpyAsync(canon, v, (size_t)vec_len(c) * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
        Level& l0 = *c->levels[0];
        launch_unpack(v, canon, l0.L, l0.C, st);
    }
}

// y = A x (mode 0) or b - A x (mode 1) on the finest level's Krylov vectors
static void vec_apply(biot_ctx* c, const double* x, const double* b, double* y, int mode, hipStream_t st) {
    if (c->sp)
        sp_apply(c, 0, x, b, y, mode, st);
    else
        launch_apply<double>(c->levels[0]->view<double>(), x, b, y, mode, st);
}

// z = M^{-1} v on the Krylov vectors of level 0 (v is not modified; z is zero on absent DoFs
// and may be used as an iterate buffer).
static void precond(biot_ctx* c, const double* v, double* z, hipStream_t st) {
    if (c->sp) {
        sp_cycle(c, 0, v, z, true, false, st);
        return;
    }
    Level& l0 = *c->levels[0];
    if (c->opts.precision == BIOT_PREC_FP64) {
        // start in the buffer that makes the last step land in z
        const bool even = buffer_moves(c->opts, 0) % 2 == 0;
        double* other = l0.x64.as<double>();
        double* res = vcycle_level<double>(c, 0, v, even ? z : other, even ? other : z, st);
        if (res != z) BIOT_HIP(hipMemcpyAsync(z, res, l0.L.len * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
        launch_convert(v, l0.b32.as<float>(), l0.L.len, st);
        float* res = vcycle_level<float>(c, 0, l0.b32.as<float>(), l0.x32.as<float>(), l0.x2_32.as<float>(), st);
        launch_convert(res, z, l0.L.len, st);
    }
}

static void alloc_fp32(biot_ctx* c, hipStream_t st) {
    for (auto& lp : c->levels) {
        Level& lv = *lp;
        if (lv.x32.p) continue;
        for (DevBuf* b : {&lv.x32, &lv.b32, &lv.r32, &lv.x2_32}) {
            b->alloc((size_t)lv.L.len * sizeof(float));
            launch_fill(b->as<float>(), lv.L.len, 0.0f, st);
        }
    }
}

// ---- FGMRES (Sec. 5.1), CGS2 Arnoldi, host Givens rotations ---------------------------------------
// Layout of the Gram-Schmidt results (device hd, host view hres), capacity M, column j:
//   [0, j+1]: pass-1 dots V_i . w (i <= j) and |w|^2 before pass 1;
//   [M+2, M+j+3]: pass-2 dots and |w|^2 after pass 1;
//   2M+5: second-pass flag;  2M+6: |w|^2 after pass 2;  2M+7: scratch
static int kslot_flag(int m) { return 2 * m + 5; }
static int kslot_n2(int m) { return 2 * m + 6; }
static int kslot_tmp(int m) { return 2 * m + 7; }
static int kslots(int m) { return 2 * m + 8; }

// The device and host memory one FGMRES solve works in.  Absent DoFs must be zero in every
// Krylov vector V_q, Z_q and in w on entry (the kernels never write them).
struct KrylovWork {
    int M = 0;                 // capacity: restart <= M; layout of the result slots
    double *V = nullptr, *Z = nullptr, *w = nullptr, *partial = nullptr;
    double *hd = nullptr, *yd = nullptr, *bpad = nullptr, *xpad = nullptr;
    double* hh = nullptr;      // device address of a mapped host mirror of hd, or nullptr
    double* hres = nullptr;    // host view of the results (kslots(M) doubles): the mirror itself,
                               // or a host array that receives a copy of hd at every synchronization
    double* hwork = nullptr;   // host: Hessenberg (M+1) x M, cs, sn (M each), g (M+1), y (M)
};
static size_t host_work_doubles(int m) { return (size_t)(m + 1) * m + 3 * (size_t)m + 1 + m; }

static void krylov_alloc(biot_ctx* c, int m, hipStream_t st) {
    if (c->krylov_m >= m) return;
    const long long len = vec_len(c);
    c->V.alloc((size_t)(m + 1) * len * sizeof(double));
    c->Z.alloc((size_t)m * len * sizeof(double));
    // absent DoFs stay zero in every Krylov vector (the kernels never write them)
    launch_fill(c->V.as<double>(), (long long)(m + 1) * len, 0.0, st);
    launch_fill(c->Z.as<double>(), (long long)m * len, 0.0, st);
    c->w.alloc((size_t)len * sizeof(double));
    launch_fill(c->w.as<double>(), len, 0.0, st);
    c->partial.alloc((size_t)RED_BLOCKS * std::max(m + 2, 4) * sizeof(double));
    c->hdev.alloc((size_t)kslots(m) * sizeof(double));
    c->ydev.alloc((size_t)(m + 1) * sizeof(double));
    c->bpad.alloc((size_t)len * sizeof(double));
    c->xpad.alloc((size_t)len * sizeof(double));
    if (c->hhost) BIOT_HIP(hipHostFree(c->hhost));
    c->hhost = nullptr;
    BIOT_HIP(hipHostMalloc((void**)&c->hhost, (size_t)kslots(m) * sizeof(double),
                           hipHostMallocMapped | hipHostMallocCoherent));
    BIOT_HIP(hipHostGetDevicePointer((void**)&c->hhost_dev, c->hhost, 0));
    c->hwork.assign(host_work_doubles(m), 0.0);
    c->krylov_m = m;
}

// the context's own workspace (allocated by krylov_alloc)
static KrylovWork context_work(biot_ctx* c) {
    KrylovWork k;
    k.M = c->krylov_m;
    k.V = c->V.as<double>();
    k.Z = c->Z.as<double>();
    k.w = c->w.as<double>();
    k.partial = c->partial.as<double>();
    k.hd = c->hdev.as<double>();
    k.yd = c->ydev.as<double>();
    k.bpad = c->bpad.as<double>();
    k.xpad = c->xpad.as<double>();
    k.hh = c->hhost_dev;
    k.hres = c->hhost;
    k.hwork = c->hwork.data();
    return k;
}

// wait for the stream; without a mapped mirror, copy the result slots to the host view first
static void sync_results(const KrylovWork& k, hipStream_t st) {
    if (!k.hh) BIOT_HIP(hipMemcpyAsync(k.hres, k.hd, (size_t)kslots(k.M) * sizeof(double), hipMemcpyDeviceToHost, st));
    BIOT_HIP(hipStreamSynchronize(st));
}

// |a|^2 (synchronizes the stream)
static double norm2_dev(const KrylovWork& k, const double* a, long long n, hipStream_t st) {
    launch_gs_dots(nullptr, 0, 0, a, n, k.partial, k.hd + kslot_tmp(k.M), k.hh ? k.hh + kslot_tmp(k.M) : nullptr,
                   nullptr, st);
    sync_results(k, st);
    return k.hres[kslot_tmp(k.M)];
}

static int fgmres(biot_ctx* c, const KrylovWork& K, const double* b_canon, double* x_canon, biot_solve_info* info,
                  hipStream_t st) {
    const long long n = vec_len(c);
    const int m = info->restart;
    const int M = K.M;                        // layout of the result slots
    if (m > M) throw ArgError{"restart exceeds the Krylov workspace"};
    double* V = K.V;
    double* Z = K.Z;
    double* w = K.w;
    double* b = K.bpad;
    double* x = K.xpad;
    double* hd = K.hd;
    double* hh = K.hh;
    const double* hres = K.hres;
    double* part = K.partial;
    vec_pack(c, b_canon, b, st);
    // the padding slots hold zeros; with x0 the free slots take the caller's initial guess
    launch_fill(x, n, 0.0, st);
    const bool warm = info->x0 == 1;
    if (warm) vec_pack(c, x_canon, x, st);
    const double bnorm = std::sqrt(norm2_dev(K, b, n, st));
    info->iters = 0;
    info->converged = 0;
    info->rel_res_true = 0;
    info->rel_res_prec = 0;
    if (!(bnorm == bnorm) || std::isinf(bnorm)) throw std::domain_error("NaN/Inf in right-hand side");
    if (bnorm == 0.0) {
        launch_fill(x, n, 0.0, st);
        vec_unpack(c, x, x_canon, st);
        info->converged = 1;
        return BIOT_OK;
    }
    const double tol = info->tol;
    // right preconditioning (flexible GMRES): the Krylov space of A M^{-1}, stopping on the true
    // residual |b - A x| <= tol |b|.  Left preconditioning: GMRES on M^{-1} A x = M^{-1} b,
    // stopping on the preconditioned residual |M^{-1}(b - A x)| <= tol |M^{-1} b| (the Z vectors
    // are not needed; the first one is scratch).
    const bool left = info->side == 1;
    const double eta2 = info->reorth > 0 ? info->reorth * info->reorth : 0.5;   // DGKS threshold, squared
    double* tmp = Z;
    double znorm = bnorm;           // the stopping test's reference norm
    double beta;
    double rtrue = bnorm;
    if (left) {
        // the cycle writes the free DoFs of its output only: w must hold zeros elsewhere
        launch_fill(w, n, 0.0, st);
        precond(c, b, w, st);
        znorm = std::sqrt(norm2_dev(K, w, n, st));
        if (!(znorm == znorm) || std::isinf(znorm)) throw std::domain_error("NaN/Inf in the preconditioned right-hand side");
        beta = znorm;
        if (warm) {
            // the preconditioned residual of the initial guess
            vec_apply(c, x, b, tmp, 1, st);
            rtrue = std::sqrt(norm2_dev(K, tmp, n, st));
            precond(c, tmp, w, st);
            beta = std::sqrt(norm2_dev(K, w, n, st));
        }
    } else if (warm) {
        // r = b - A x0
        vec_apply(c, x, b, w, 1, st);
        beta = rtrue = std::sqrt(norm2_dev(K, w, n, st));
    } else {
        // r = b - A x  (x = 0 -> r = b)
        BIOT_HIP(hipMemcpyAsync(w, b, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        beta = bnorm;
    }
    if (!(beta == beta) || std::isinf(beta)) throw std::domain_error("NaN/Inf in the initial residual");
    // host arrays: Hessenberg (m + 1) x m, rotations, right-hand side and solution of the LS problem
    double* H = K.hwork;
    double* cs = H + (size_t)(m + 1) * m;
    double* sn = cs + m;
    double* g = sn + m;
    double* y = g + m + 1;
    // mirrors of the flag (and, unfused, of the pass-2 dots) for the host's reads
    double* hflag = hh ? hh + kslot_flag(M) : nullptr;
    int it = 0;
    while (true) {
        if (beta <= tol * znorm) {
            info->converged = 1;
            break;
        }
        if (it >= info->maxit) break;
        // V_0 = r / beta
        launch_scale(V, w, n, 1.0 / beta, st);
        std::fill(H, H + (size_t)(m + 1) * m, 0.0);
        std::fill(g, g + m + 1, 0.0);
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double* vj = V + (size_t)j * n;
            double* zj = Z + (size_t)j * n;
            if (left) {
                // w = M^{-1} A v_j
                vec_apply(c, vj, nullptr, tmp, 0, st);
                precond(c, tmp, w, st);
            } else {
                precond(c, vj, zj, st);
                // Arnoldi on the shifted vector w = v_j - A z_j (A z_j = v_j - w): with a good
                // preconditioner A z_j is close to v_j, so A z_j itself lies almost entirely in the
                // Krylov basis and orthogonalizing it cancels nearly everything, while the shifted
                // vector keeps the part that is new.  Its coefficients are h'_i = delta_ij - h_i and
                // the orthogonalized remainder is -h_{j+1,j} v_{j+1}.
                vec_apply(c, zj, vj, w, 1, st);
            }
            // CGS with a second pass when the first one cancels (|w| drops below |w_0| / sqrt 2).
            // Pass one's update also forms pass two's dot products (V is read once for both), so
            // the second pass costs one more update only when it runs.
            const int nv = j + 1;
            const bool fused = nv <= GS_FUSED;
            launch_gs_dots(V, n, nv, w, n, part, hd, hh, nullptr, st);
            if (fused) {
                launch_gs_update_dots(w, V, n, nv, hd, n, part, hd + M + 2, hh ? hh + M + 2 : nullptr, hd + nv,
                                      hd + kslot_flag(M), hflag, st, eta2);
            } else {
                launch_gs_update(w, V, n, nv, hd, n, part, hd + M + 2 + nv, hd + nv, hd + kslot_flag(M),
                                 hh ? hh + M + 2 + nv : nullptr, nullptr, st, eta2);
                launch_gs_dots(V, n, nv, w, n, part, hd + M + 2, hh ? hh + M + 2 : nullptr, hd + kslot_flag(M), st);
                if (hflag)
                    BIOT_HIP(hipMemcpyAsync(hflag, hd + kslot_flag(M), sizeof(double), hipMemcpyDeviceToDevice, st));
            }
            launch_gs_update(w, V, n, nv, hd + M + 2, n, part, hd + kslot_n2(M), nullptr, nullptr,
                             hh ? hh + kslot_n2(M) : nullptr, hd + kslot_flag(M), st);
            launch_normalize(V + (size_t)nv * n, w, n, hd + M + 2 + nv, hd + kslot_n2(M), hd + kslot_flag(M), st);
            check_stream_error();
            sync_results(K, st);
            const bool second = hres[kslot_flag(M)] != 0.0;
            const double hn = std::sqrt(second ? hres[kslot_n2(M)] : hres[M + 2 + nv]);
            if (left) {
                for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hres[i] + (second ? hres[M + 2 + i] : 0.0);
                H[(size_t)(j + 1) * m + j] = hn;
            } else {
                for (int i = 0; i <= j; ++i)
                    H[(size_t)i * m + j] = (i == j ? 1.0 : 0.0) - (hres[i] + (second ? hres[M + 2 + i] : 0.0));
                // v_{j+1} = w / |w| is minus the direction of the unshifted remainder
                H[(size_t)(j + 1) * m + j] = -hn;
            }
            for (int i = 0; i <= j + 1; ++i)
                if (!(H[(size_t)i * m + j] == H[(size_t)i * m + j])) throw std::domain_error("NaN in Arnoldi");
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            const double den = std::hypot(a, bb);
            cs[j] = a / den;
            sn[j] = bb / den;
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            k = j + 1;
            if (std::fabs(g[j + 1]) <= tol * znorm || it >= info->maxit || hn == 0.0) break;
        }
        // y = H^{-1} g (upper triangular k x k), x += Z y
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int q = i + 1; q < k; ++q) s -= H[(size_t)i * m + q] * y[q];
            y[i] = s / H[(size_t)i * m + i];
        }
        BIOT_HIP(hipMemcpyAsync(K.yd, y, k * sizeof(double), hipMemcpyHostToDevice, st));
        launch_lincomb_add(x, left ? V : Z, n, k, K.yd, n, st);
        // true residual; left: the preconditioned residual that restarts the iteration
        if (left) {
            vec_apply(c, x, b, tmp, 1, st);
            rtrue = std::sqrt(norm2_dev(K, tmp, n, st));
            precond(c, tmp, w, st);
            beta = std::sqrt(norm2_dev(K, w, n, st));
        } else {
            vec_apply(c, x, b, w, 1, st);
            beta = rtrue = std::sqrt(norm2_dev(K, w, n, st));
        }
        if (!(beta == beta) || !(rtrue == rtrue)) throw std::domain_error("NaN in residual");
    }
    info->iters = it;
    info->rel_res_true = rtrue / bnorm;
    info->rel_res_prec = left ? beta / znorm : 0.0;
    vec_unpack(c, x, x_canon, st);
    check_stream_error();
    return info->converged ? BIOT_OK : BIOT_NOT_CONVERGED;
}

// ---- workspace without allocation -------------------------------------------------------------
// A fixed device array that biot_solve_noalloc carves its Krylov workspace from.  Host code never
// passes the array's name to a kernel: it uses the address hipGetSymbolAddress returns on each
// device (resolved once per device at biot_assemble, or at the entry point's first call there).
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_MAX_RESTART = 32;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) double scratch[NOALLOC_BYTES / sizeof(double)];
static double* g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mutex;

// the scratch address on the current device (resolves it on first use there)
static double* scratch_address() {
    int dev = 0;
    BIOT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) throw ArgError{"device index beyond the scratch table"};
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        BIOT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)"};
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    return g_scratch_ptr[dev];
}

static size_t round256(size_t doubles) { return (doubles + 31) / 32 * 32; }

// doubles of scratch a solve with restart m on a padded length len needs
static size_t noalloc_doubles(long long len, int m) {
    return round256((size_t)(m + 1) * len) + round256((size_t)m * len) + 3 * round256((size_t)len) +
           round256((size_t)RED_BLOCKS * std::max(m + 2, 4)) + round256((size_t)kslots(m)) + round256((size_t)m + 1);
}

// carve the workspace out of the scratch array; V and Z are cleared (a previous call, possibly
// with another layout, may have left values at this layout's absent DoFs)
static KrylovWork scratch_work(double* base, long long len, int m, double* hres, double* hwork, hipStream_t st) {
    KrylovWork k;
    k.M = m;
    size_t off = 0;
    auto take = [&](size_t cnt) {
        double* p = base + off;
        off += round256(cnt);
        return p;
    };
    k.V = take((size_t)(m + 1) * len);
    k.Z = take((size_t)m * len);
    k.w = take(len);
    k.bpad = take(len);
    k.xpad = take(len);
    k.partial = take((size_t)RED_BLOCKS * std::max(m + 2, 4));
    k.hd = take(kslots(m));
    k.yd = take((size_t)m + 1);
    launch_fill(k.V, (long long)(m + 1) * len, 0.0, st);
    launch_fill(k.Z, (long long)m * len, 0.0, st);
    launch_fill(k.w, len, 0.0, st);
    k.hh = nullptr;
    k.hres = hres;
    k.hwork = hwork;
    return k;
}

}  // namespace biot

// =================================================================================================
// C ABI
// =================================================================================================
template <typename F>
static int guarded(F&& f) {
    try {
        return f();
    } catch (const ArgError& e) {
        set_error(e.msg);
        return BIOT_ERR_ARG;
    } catch (const SingularError& e) {
        set_error(e.msg);
        return BIOT_ERR_SINGULAR;
    } catch (const HipError& e) {
        set_error(std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
        return BIOT_ERR_HIP;
    } catch (const std::bad_alloc&) {
        (void)hipGetLastError();
        set_error("device or host allocation failed");
        return BIOT_ERR_OOM;
    } catch (const std::domain_error& e) {
        set_error(e.what());
        return BIOT_ERR_NAN;
    } catch (const std::exception& e) {
        set_error(e.what());
        return BIOT_ERR_ARG;
    } catch (...) {
        set_error("unknown failure");
        return BIOT_ERR_ARG;
    }
}

static hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

static void require(bool ok, const char* msg) {
    if (!ok) throw ArgError{msg};
}

static void require_ctx(biot_ctx* c) { require(c != nullptr, "null context"); }

static void require_hierarchy(biot_ctx* c) {
    require_ctx(c);
    require(c->have_hierarchy, "biot_setup_hierarchy has not been called");
}

static int num_levels(biot_ctx* c) { return c->sp ? (int)c->sp->lv.size() : (int)c->levels.size(); }

static void require_level(biot_ctx* c, int level) {
    require_ctx(c);
    require(level >= 0 && level < num_levels(c), "level out of range");
}

static void require_structured(biot_ctx* c, const char* what) {
    if (c->sp) throw ArgError{std::string(what) + " is not available with bc = BIOT_BC_TERZAGHI"};
}

extern "C" {

int biot_assemble(const biot_problem* prob, void* stream, biot_ctx** out) {
    if (out) *out = nullptr;
    return guarded([&]() {
        require(prob != nullptr && out != nullptr, "null argument");
        const int n = prob->n;
        require(prob->bc == BIOT_BC_DIRICHLET || prob->bc == BIOT_BC_TERZAGHI, "bc: BIOT_BC_DIRICHLET or BIOT_BC_TERZAGHI");
        const bool sparse = prob->bc != BIOT_BC_DIRICHLET;
        require(n >= 4 && n <= 8192 && (n & (n - 1)) == 0, "n must be a power of two in [4, 8192]");
        require(!sparse || n <= 256, "bc = BIOT_BC_TERZAGHI: n <= 256");
        require(prob->mu > 0 && prob->lambda >= 0, "need mu > 0 and lambda >= 0");
        if (sparse)
            require(prob->inv_M >= 0 && std::isfinite(prob->inv_M), "need 0 <= 1/M < inf");
        else
            require(prob->inv_M > 0 && std::isfinite(prob->inv_M), "need 0 < 1/M < inf");
        require(prob->mu_f > 0 && prob->tau > 0, "need mu_f > 0 and tau > 0");
        require(std::isfinite(prob->alpha) && std::isfinite(prob->lambda) && std::isfinite(prob->mu),
                "non-finite parameter");
        require(prob->K_tri != nullptr || (prob->K_scalar > 0 && std::isfinite(prob->K_scalar) &&
                                           std::isfinite(1.0 / prob->K_scalar)),
                "need finite K_scalar > 0 (with finite 1/K) when K_tri is NULL");
        // the no-allocation solve's scratch address on this device (set-up of the library on a
        // device; a failure here is reported by biot_solve_noalloc, which tries again)
        try {
            (void)scratch_address();
        } catch (const HipError&) {
            (void)hipGetLastError();
        }
        std::unique_ptr<biot_ctx> c(new biot_ctx);
        c->n = n;
        c->phys = PhysParams{prob->lambda, prob->mu, prob->alpha, prob->inv_M, prob->mu_f, prob->tau};
        c->K_scalar = prob->K_scalar;
        c->K_uniform = (prob->K_tri == nullptr);
        hipStream_t st = S(stream);
        c->kcheck.alloc(sizeof(int));
        if (prob->K_tri) check_field(c.get(), prob->K_tri, 0, st);
        if (sparse) {
            c->sp.reset(new SpHier);
            c->sp->bc = prob->bc;
            c->sp->lv.emplace_back(new SpLevel);
            sp_level_alloc(*c->sp->lv[0], n, prob->bc, c->phys, st);
            sp_assemble(c.get(), prob->K_tri, 0, st);
            check_stream_error();
            BIOT_HIP(hipStreamSynchronize(st));
            *out = c.release();
            return BIOT_OK;
        }
        c->levels.emplace_back(new Level);
        level_alloc(*c->levels[0], n, st);
        level_stencil(*c->levels[0], c->phys, st);
        launch_kinv_from_K(prob->K_tri, prob->K_scalar, c->levels[0]->kinv64.as<double>(), c->levels[0]->L, st);
        launch_convert(c->levels[0]->kinv64.as<double>(), c->levels[0]->kinv32.as<float>(),
                       2 * c->levels[0]->L.plane, st);
        // local RT0 mass blocks for the adjoint: the K-tagged stencil entries of one triangle
        {
            std::vector<double> m(18, 0.0);
            // L(i,j): local order D(i,j), V(i,j), H(i,j); U(i,j): H(i,j+1), D(i,j), V(i+1,j)
            const int tl[3] = {T_WD, T_WV, T_WH}, tu[3] = {T_WH, T_WD, T_WV};
            const int lo_i[2][3] = {{0, 0, 0}, {0, 0, 1}}, lo_j[2][3] = {{0, 0, 0}, {1, 0, 0}};
            for (int u = 0; u < 2; ++u)
                for (int a = 0; a < 3; ++a)
                    for (int bq = 0; bq < 3; ++bq) {
                        const int ta = u ? tu[a] : tl[a], tb = u ? tu[bq] : tl[bq];
                        for (auto& e : c->levels[0]->st_host) {
                            if (e.ktri != u || e.out_t != ta || e.in_t != tb) continue;
                            // entry anchored at row slot s_a; triangle at s_a + (kdi, kdj) must be (0,0)
                            if (lo_i[u][a] + e.kdi != 0 || lo_j[u][a] + e.kdj != 0) continue;
                            if (e.di != lo_i[u][bq] - lo_i[u][a] || e.dj != lo_j[u][bq] - lo_j[u][a]) continue;
                            m[u * 9 + a * 3 + bq] += e.coef;
                        }
                    }
            upload(c->mloc, m, st);
        }
        check_stream_error();
        BIOT_HIP(hipStreamSynchronize(st));
        *out = c.release();
        return BIOT_OK;
    });
}

int biot_setup_hierarchy(biot_ctx* c, const biot_mg_opts* o, void* stream) {
    return guarded([&]() {
        require_ctx(c);
        require(o != nullptr, "null options");
        require(o->levels >= 2, "need at least 2 levels");
        require((c->n >> (o->levels - 1)) >= 2 && ((c->n >> (o->levels - 1)) << (o->levels - 1)) == c->n,
                "coarsest mesh n >> (levels-1) must be >= 2");
        require(o->smoother == BIOT_SMOOTHER_VANKA || o->smoother == BIOT_SMOOTHER_BSR, "unknown smoother");
        require(o->nu1 >= 0 && o->nu1 <= 16 && o->nu2 >= 0 && o->nu2 <= 16 && o->nu1 + o->nu2 >= 1,
                "nu1, nu2 in [0, 16], nu1 + nu2 >= 1");
        require(o->precision == BIOT_PREC_FP64 || o->precision == BIOT_PREC_FP32_SMOOTHER ||
                    o->precision == BIOT_PREC_FP32_PATCH, "unknown precision");
        require(std::isfinite(o->omega) && o->omega > 0, "omega must be positive");
        require(o->smoother != BIOT_SMOOTHER_BSR || (std::isfinite(o->omega_J) && o->omega_J > 0),
                "BSR needs omega_J > 0");
        require(o->schur_sweeps >= 0 && o->schur_sweeps <= 64, "schur_sweeps in [0, 64]");
        require(o->gamma >= 0 && o->gamma <= 4, "gamma (cycle index) in [0, 4]");
        require(o->gamma_from >= 0 && o->gamma_from < o->levels, "gamma_from in [0, levels)");
        require(o->fcycle == 0 || o->fcycle == 1, "fcycle: 0 (W-cycle) or 1 (F-cycle)");
        require(o->gamma_to >= 0 && o->gamma_to < o->levels, "gamma_to in [0, levels)");
        require(o->vanka_colors == 0 || o->vanka_colors == 3 || o->vanka_colors == 4,
                "vanka_colors: 0 (additive), 3 or 4");
        require(o->schur_sweeps <= 1 || (std::isfinite(o->omega_S) && o->omega_S > 0 && o->omega_S <= 1),
                "Schur sweeps need omega_S in (0, 1]");
        require(o->schur_cg >= 0 && o->schur_cg <= 64, "schur_cg in [0, 64]");
        require(o->schur_cg == 0 || o->schur_sweeps <= 1, "schur_cg and schur_sweeps > 1 exclude each other");
        require(std::isfinite(o->vanka_shift) && o->vanka_shift >= 0, "vanka_shift >= 0");
        require(o->csr_below >= 0, "csr_below >= 0");
        require(o->additive_levels >= 0 && o->additive_levels < o->levels, "additive_levels in [0, levels)");
        require(std::isfinite(o->omega_additive) && o->omega_additive >= 0, "omega_additive >= 0");
        require(o->csr_below == 0 || o->smoother == BIOT_SMOOTHER_VANKA, "csr_below: Vanka only");
        const int nc = c->n >> (o->levels - 1);
        require(nc <= 16, "coarsest mesh must have at most 16 cells per side (dense direct solve)");
        hipStream_t st = S(stream);
        if (c->sp) {
            require(o->smoother == BIOT_SMOOTHER_VANKA && o->vanka_colors == 0,
                    "bc = BIOT_BC_TERZAGHI: additive Vanka only (smoother VANKA, vanka_colors 0)");
            require(o->precision == BIOT_PREC_FP64, "bc = BIOT_BC_TERZAGHI: precision BIOT_PREC_FP64 only");
            // with 1/M = 0 the pressure constant on the star of an interior vertex is in the null
            // space of its patch matrix (the patch velocities carry no net flux of it)
            require(c->phys.inv_M > 0 || o->vanka_shift > 0,
                    "1/M = 0: the interior Vanka patch matrices are singular; set vanka_shift > 0");
            sp_setup(c, o, st);
            return BIOT_OK;
        }
        require(o->vanka_shift == 0, "vanka_shift is available with bc = BIOT_BC_TERZAGHI only");
        c->have_hierarchy = false;
        // (re)build levels 1..L-1
        c->levels.resize(1);
        for (int l = 1; l < o->levels; ++l) {
            c->levels.emplace_back(new Level);
            level_alloc(*c->levels[l], c->n >> l, st);
            level_stencil(*c->levels[l], c->phys, st);
        }
        for (auto& lv : c->levels) level_patch_data(*lv, c->K_uniform, 1.0 / c->K_scalar, st);
        {
            std::vector<double> w(NPWEIGHTS);
            build_prolong_weights(w.data());
            upload(c->pw64, w, st);
            std::vector<float> wf(w.begin(), w.end());
            upload(c->pw32, wf, st);
        }
        for (size_t l = 1; l < c->levels.size(); ++l)
            launch_kinv_coarsen(c->levels[l - 1]->kinv64.as<double>(), c->levels[l - 1]->L,
                                c->levels[l]->kinv64.as<double>(), c->levels[l]->L, st);
        for (auto& lv : c->levels)
            launch_convert(lv->kinv64.as<double>(), lv->kinv32.as<float>(), 2 * lv->L.plane, st);
        levels_factors(c, st);
        c->opts = *o;
        if (c->opts.gamma < 1) c->opts.gamma = 1;
        if (o->precision != BIOT_PREC_FP64) alloc_fp32(c, st);
        for (auto& lp : c->levels) lp->patch32 = o->precision == BIOT_PREC_FP32_PATCH;
        if (o->smoother == BIOT_SMOOTHER_BSR) levels_bsr(c, st);
        coarse_setup(c, st);
        coarse_factor(c, st);
        small_setup(c, st);
        check_stream_error();
        BIOT_HIP(hipStreamSynchronize(st));
        c->have_hierarchy = true;
        return BIOT_OK;
    });
}

int biot_vcycle(biot_ctx* c, const double* r, double* z, void* stream) {
    return guarded([&]() {
        require_hierarchy(c);
        require(r && z && r != z, "r and z must be distinct non-null device pointers");
        hipStream_t st = S(stream);
        if (c->sp) {
            sp_cycle(c, 0, r, z, true, false, st);
            check_stream_error();
            return BIOT_OK;
        }
        Level& l0 = *c->levels[0];
        launch_pack(r, l0.b64.as<double>(), l0.L, l0.C, st);
        precond(c, l0.b64.as<double>(), l0.t64.as<double>(), st);
        launch_unpack(l0.t64.as<double>(), z, l0.L, l0.C, st);
        check_stream_error();
        return BIOT_OK;
    });
}

int biot_solve(biot_ctx* c, const double* b, double* x, biot_solve_info* info, void* stream) {
    return guarded([&]() {
        require_hierarchy(c);
        require(b && x && b != x, "b and x must be distinct non-null device pointers");
        require(info != nullptr, "null info");
        require(info->restart >= 1 && info->restart <= 200, "restart in [1, 200]");
        require(info->maxit >= 0, "maxit >= 0");
        require(info->tol >= 0 && std::isfinite(info->tol), "tol >= 0");
        require(info->side == 0 || info->side == 1, "side: 0 (right) or 1 (left)");
        require(info->reorth >= 0 && info->reorth <= 1, "reorth (the DGKS eta) in [0, 1]");
        require(info->x0 == 0 || info->x0 == 1, "x0: 0 (zero initial guess) or 1 (x holds it)");
        krylov_alloc(c, info->restart, S(stream));
        return fgmres(c, context_work(c), b, x, info, S(stream));
    });
}

int biot_solve_noalloc(biot_ctx* c, const double* b, double* x, biot_solve_info* info, void* stream) {
    return guarded([&]() {
        require_hierarchy(c);
        require(b && x && b != x, "b and x must be distinct non-null device pointers");
        require(info != nullptr, "null info");
        require(info->restart >= 1 && info->restart <= NOALLOC_MAX_RESTART,
                "biot_solve_noalloc: restart in [1, 32]");
        require(info->maxit >= 0, "maxit >= 0");
        require(info->tol >= 0 && std::isfinite(info->tol), "tol >= 0");
        require(info->side == 0 || info->side == 1, "side: 0 (right) or 1 (left)");
        require(info->reorth >= 0 && info->reorth <= 1, "reorth (the DGKS eta) in [0, 1]");
        require(info->x0 == 0 || info->x0 == 1, "x0: 0 (zero initial guess) or 1 (x holds it)");
        require_structured(c, "biot_solve_noalloc");
        const long long len = c->levels[0]->L.len;
        const size_t need = noalloc_doubles(len, info->restart) * sizeof(double);
        if (need > NOALLOC_BYTES)
            throw ArgError{"biot_solve_noalloc: mesh n = " + std::to_string(c->n) + " with restart " +
                           std::to_string(info->restart) + " needs " + std::to_string(need >> 20) +
                           " MiB of workspace, more than the fixed 64 MiB"};
        hipStream_t st = S(stream);
        double* base = scratch_address();
        double hres[2 * NOALLOC_MAX_RESTART + 8];
        double hwork[(NOALLOC_MAX_RESTART + 1) * NOALLOC_MAX_RESTART + 4 * NOALLOC_MAX_RESTART + 1];
        return fgmres(c, scratch_work(base, len, info->restart, hres, hwork, st), b, x, info, st);
    });
}

int biot_apply_operator(biot_ctx* c, int level, const double* x, double* y, void* stream) {
    return guarded([&]() {
        require_level(c, level);
        require(x && y && x != y, "x and y must be distinct non-null device pointers");
        hipStream_t st = S(stream);
        if (c->sp) {
            sp_apply(c, level, x, nullptr, y, 0, st);
            check_stream_error();
            return BIOT_OK;
        }
        Level& lv = *c->levels[level];
        launch_pack(x, lv.t64.as<double>(), lv.L, lv.C, st);
        launch_apply<double>(lv.view<double>(), lv.t64.as<double>(), nullptr, lv.r64.as<double>(), 0, st);
        launch_unpack(lv.r64.as<double>(), y, lv.L, lv.C, st);
        check_stream_error();
        return BIOT_OK;
    });
}

int biot_smooth(biot_ctx* c, int level, double* x, const double* b, void* stream) {
    return guarded([&]() {
        require_hierarchy(c);
        require_level(c, level);
        require(level < num_levels(c) - 1, "no smoother on the coarsest level");
        require(x && b && (const double*)x != b, "x and b must be distinct non-null device pointers");
        hipStream_t st = S(stream);
        if (c->sp) {
            sp_smooth(c, level, x, b, false, st);
            check_stream_error();
            return BIOT_OK;
        }
        Level& lv = *c->levels[level];
        launch_pack(x, lv.x64.as<double>(), lv.L, lv.C, st);
        launch_pack(b, lv.b64.as<double>(), lv.L, lv.C, st);
        const bool vanka = c->opts.smoother == BIOT_SMOOTHER_VANKA;
        if (c->opts.precision == BIOT_PREC_FP64) {
            double* x0 = lv.x64.as<double>();
            double* res = relax<double>(c, level, x0, lv.b64.as<double>(), vanka ? lv.x2_64.as<double>() : x0, x0, st);
            launch_unpack(res, x, lv.L, lv.C, st);
        } else {
            float* x0 = lv.x32.as<float>();
            launch_convert(lv.x64.as<double>(), x0, lv.L.len, st);
            launch_convert(lv.b64.as<double>(), lv.b32.as<float>(), lv.L.len, st);
            float* res = relax<float>(c, level, x0, lv.b32.as<float>(), vanka ? lv.x2_32.as<float>() : x0, x0, st);
            launch_convert(res, lv.x64.as<double>(), lv.L.len, st);
            launch_unpack(lv.x64.as<double>(), x, lv.L, lv.C, st);
        }
        check_stream_error();
        return BIOT_OK;
    });
}

int biot_restrict(biot_ctx* c, int level, const double* r_f, double* r_c, void* stream) {
    return guarded([&]() {
        require_hierarchy(c);
        require_level(c, level);
        require(level + 1 < num_levels(c), "no coarser level");
        require(r_f && r_c, "null pointer");
        hipStream_t st = S(stream);
        if (c->sp) {
            const SpLevel& F = *c->sp->lv[level];
            const SpLevel& C = *c->sp->lv[level + 1];
            launch_csr_mv(C.N, F.rptr.as<int>(), F.rcol.as<int>(), F.rval.as<double>(), r_f, nullptr, r_c, 1.0, 0.0, st);
            check_stream_error();
            return BIOT_OK;
        }
        Level& lf = *c->levels[level];
        Level& lc = *c->levels[level + 1];
        launch_pack(r_f, lf.t64.as<double>(), lf.L, lf.C, st);
        launch_restrict<double>(lf.L, lc.L, lf.t64.as<double>(), lc.t64.as<double>(), c->pw64.as<double>(), st);
        launch_unpack(lc.t64.as<double>(), r_c, lc.L, lc.C, st);
        check_stream_error();
        return BIOT_OK;
    });
}

int biot_prolong_add(biot_ctx* c, int level, const double* x_c, double* x_f, void* stream) {
    return guarded([&]() {
        require_hierarchy(c);
        require_level(c, level);
        require(level + 1 < num_levels(c), "no coarser level");
        require(x_c && x_f && x_c != (const double*)x_f, "x_c and x_f must be distinct non-null device pointers");
        hipStream_t st = S(stream);
        if (c->sp) {
            const SpLevel& F = *c->sp->lv[level];
            launch_csr_mv(F.N, F.pptr.as<int>(), F.pcol.as<int>(), F.pval.as<double>(), x_c, x_f, x_f, 1.0, 1.0, st);
            check_stream_error();
            return BIOT_OK;
        }
        Level& lf = *c->levels[level];
        Level& lc = *c->levels[level + 1];
        launch_pack(x_c, lc.t64.as<double>(), lc.L, lc.C, st);
        launch_pack(x_f, lf.t64.as<double>(), lf.L, lf.C, st);
        launch_prolong_add<double>(lf.L, lc.L, lc.t64.as<double>(), lf.t64.as<double>(), c->pw64.as<double>(), st);
        launch_unpack(lf.t64.as<double>(), x_f, lf.L, lf.C, st);
        check_stream_error();
        return BIOT_OK;
    });
}

// re-assembly for a new per-triangle field: mode 0 permeabilities, mode 1 log-permeabilities
static int update_perm(biot_ctx* c, const double* field, int mode, void* stream) {
    require_ctx(c);
    require(field != nullptr, mode == 0 ? "null K" : "null theta");
    hipStream_t st = S(stream);
    check_field(c, field, mode, st);
    c->K_uniform = false;
    if (c->sp) {
        sp_assemble(c, field, mode, st);
        if (c->have_hierarchy) sp_factor(c, st);
        check_stream_error();
        return BIOT_OK;
    }
    levels_kinv(c, field, st, mode);
    if (c->have_hierarchy) levels_factors(c, st);
    if (c->have_hierarchy && c->opts.smoother == BIOT_SMOOTHER_BSR) levels_bsr(c, st);
    if (c->have_hierarchy) coarse_factor(c, st);
    if (c->have_hierarchy && c->small) small_refresh(c, st);
    check_stream_error();
    return BIOT_OK;
}

int biot_update_K(biot_ctx* c, const double* K_tri, void* stream) {
    return guarded([&]() { return update_perm(c, K_tri, 0, stream); });
}

int biot_update_logK(biot_ctx* c, const double* theta_tri, void* stream) {
    return guarded([&]() { return update_perm(c, theta_tri, 1, stream); });
}

int biot_grad_logK(biot_ctx* c, const double* x, const double* lam, double* g_tri, void* stream) {
    return guarded([&]() {
        require_ctx(c);
        require(x && lam && g_tri, "null pointer");
        require_structured(c, "biot_grad_logK");
        hipStream_t st = S(stream);
        Level& l0 = *c->levels[0];
        launch_pack(x, l0.t64.as<double>(), l0.L, l0.C, st);
        launch_pack(lam, l0.r64.as<double>(), l0.L, l0.C, st);
        launch_grad_logK(l0.L, l0.t64.as<double>(), l0.r64.as<double>(), l0.kinv64.as<double>(),
                         c->mloc.as<double>(), g_tri, st);
        check_stream_error();
        return BIOT_OK;
    });
}

int biot_export_layout(biot_ctx* c, int* counts, int* patch_table, void* stream) {
    return guarded([&]() {
        require_ctx(c);
        hipStream_t st = S(stream);
        if (c->sp) {
            require(patch_table == nullptr, "bc = BIOT_BC_TERZAGHI: the patch table is not exported");
            const FreeMap& m = c->sp->lv[0]->map;
            if (counts) {
                counts[0] = c->n;
                counts[1] = m.N;
                for (int t = 0; t < NTYPES; ++t) counts[2 + t] = (int)m.block[t];
            }
            return BIOT_OK;
        }
        Level& l0 = *c->levels[0];
        if (counts) {
            counts[0] = c->n;
            counts[1] = (int)l0.C.off[NTYPES];
            for (int t = 0; t < NTYPES; ++t) counts[2 + t] = (int)l0.C.size[t];
        }
        if (patch_table) {
            const size_t rows = (size_t)(c->n + 1) * (c->n + 1) - 2;
            DevBuf d;
            d.alloc(rows * PATCH * sizeof(int));
            launch_patch_table(l0.L, l0.C, d.as<int>(), st);
            check_stream_error();
            BIOT_HIP(hipMemcpyAsync(patch_table, d.p, rows * PATCH * sizeof(int), hipMemcpyDeviceToHost, st));
            BIOT_HIP(hipStreamSynchronize(st));
        }
        return BIOT_OK;
    });
}

int biot_kernel_timing(biot_ctx* c, int enable, int level, double* out, void* stream) {
    return guarded([&]() {
        require_level(c, level);
        require_structured(c, "biot_kernel_timing");
        hipStream_t st = S(stream);
        if (enable) {
            c->prof_on = true;
            c->prof_level = level;
            c->prof_used[0] = c->prof_used[1] = 0;
            return BIOT_OK;
        }
        c->prof_on = false;
        BIOT_HIP(hipStreamSynchronize(st));
        double tot[2] = {0, 0};
        for (int k = 0; k < 2; ++k)
            for (size_t q = 0; q + 1 < c->prof_used[k]; q += 2) {
                float ms = 0;
                BIOT_HIP(hipEventElapsedTime(&ms, c->prof_ev[k][q], c->prof_ev[k][q + 1]));
                tot[k] += ms;
            }
        if (out) {
            out[0] = tot[0];
            out[1] = (double)(c->prof_used[0] / 2);
            out[2] = tot[1];
            out[3] = (double)(c->prof_used[1] / 2);
        }
        c->prof_used[0] = c->prof_used[1] = 0;
        return BIOT_OK;
    });
}

void biot_destroy(biot_ctx* c) { delete c; }

const char* biot_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
