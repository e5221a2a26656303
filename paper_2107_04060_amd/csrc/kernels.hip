// Device kernels of the RQ Biot multigrid for gfx950 (CDNA4, 64-wide wavefronts).
//
// Vector plumbing (canonical <-> padded layout, precision), the operator (Sec. 2.1 block_form,
// 2.3 block_form_rq, Appendix A), the coarsest direct solve (Sec. 5.1), per-level 1/K, the
// adjoint gradient and the layout export.  The relaxation, transfer and Krylov kernels sit in
// vanka.hip, bsr.hip, transfer.hip and krylov.hip.
#include "kernels.h"
#include "patch_solve.h"
#include "structure.h"
#include "tile.h"

#include <type_traits>
#include <utility>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace biot {

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

template <typename T>
__global__ void k_add(T* __restrict__ y, const T* __restrict__ x, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) y[i] += x[i];
}

template <typename T>
void launch_add(T* y, const T* x, long long n, hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_add<T>, dim3(blocks), dim3(256), 0, st, y, x, n);
}
template void launch_add<double>(double*, const double*, long long, hipStream_t);
template void launch_add<float>(float*, const float*, long long, hipStream_t);

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
// coarsest level: dense inverse applied one row per wave (Sec. 5.1 direct solve)
// =========================================================================================
// Rows of up to CS_RMAX x 64 entries (the 16 x 16 coarsest mesh has 2434) are loaded whole into
// registers first, every load of a lane in flight at once and before the right-hand side is
// staged, so the row's latency overlaps the staging; longer rows go through the loop.  The
// partial sums take the same entries in the same order either way.
constexpr int CS_RMAX = 40;
template <typename T, bool REG>
__global__ __launch_bounds__(256) void k_coarse_solve(const double* __restrict__ Ainv, int N,
                                                      const int* __restrict__ idx, const T* __restrict__ b,
                                                      T* __restrict__ x) {
    extern __shared__ double bb[];
    // one row per wave: the lanes read consecutive entries of the row into eight partial sums
    // (entry lane + 64 u goes to sum u mod 8), then a butterfly sum
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const double* row = Ainv + (long long)(k < N ? k : N - 1) * N;
    double rv[REG ? CS_RMAX : 1];
    if constexpr (REG) {
#pragma unroll
        for (int u = 0; u < CS_RMAX; ++u) rv[u] = lane + u * 64 < N ? row[lane + u * 64] : 0.0;
    }
    for (int q = threadIdx.x; q < N; q += blockDim.x) bb[q] = (double)b[idx[q]];
    __syncthreads();
    if (k >= N) return;
    double ps[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if constexpr (REG) {
#pragma unroll
        for (int u = 0; u < CS_RMAX; ++u)
            if (lane + u * 64 < N) ps[u % 8] += rv[u] * bb[lane + u * 64];
    } else {
        int l = lane;
        for (; l + 7 * 64 < N; l += 8 * 64) {
#pragma unroll
            for (int u = 0; u < 8; ++u) ps[u] += row[l + u * 64] * bb[l + u * 64];
        }
        for (int u = 0; l < N; l += 64, ++u) ps[u] += row[l] * bb[l];
    }
    double s = ((ps[0] + ps[1]) + (ps[2] + ps[3])) + ((ps[4] + ps[5]) + (ps[6] + ps[7]));
    s = wave_sum(s);
    if (lane == 0) x[idx[k]] = (T)s;
}

template <typename T>
void launch_coarse_solve(const double* Ainv, int N, const int* idx, const T* b, T* x, hipStream_t st) {
    if (N <= CS_RMAX * 64)
        hipLaunchKernelGGL((k_coarse_solve<T, true>), dim3((N + 3) / 4), dim3(256), N * sizeof(double), st, Ainv, N, idx,
                           b, x);
    else
        hipLaunchKernelGGL((k_coarse_solve<T, false>), dim3((N + 3) / 4), dim3(256), N * sizeof(double), st, Ainv, N,
                           idx, b, x);
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

// Gauss-Jordan inversion with partial pivoting, one pivot column per pair of launches (the
// elimination spreads over the whole device, so a coarsest mesh of 16 x 16, N = 2434, inverts in
// a fraction of a second); M is destroyed.  status: 0, or 1 once a zero pivot column is met
// (every later launch then returns at once).
__global__ void k_gj_identity(double* __restrict__ Inv, int N, int* __restrict__ status) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) *status = 0;
    if (q < (long long)N * N) Inv[q] = ((q / N) == (q % N)) ? 1.0 : 0.0;
}

// column c: the pivot row (largest |M[r][c]|, r >= c, the lowest index among equals), the swap
// of rows c and pivot in M and Inv, the scaling of row c by 1 / pivot, and column c of M into
// fcol (the elimination factors)
__global__ __launch_bounds__(256) void k_gj_pivot(double* __restrict__ M, double* __restrict__ Inv, int N, int c,
                                                  double* __restrict__ fcol, int* __restrict__ status) {
    __shared__ double rv[256];
    __shared__ int ri[256];
    __shared__ int piv;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (*status) return;
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
}

// every row r != c: row_r -= fcol[r] row_c, in M and Inv (row c is only read)
__global__ __launch_bounds__(256) void k_gj_eliminate(double* __restrict__ M, double* __restrict__ Inv, int N, int c,
                                                      const double* __restrict__ fcol, const int* __restrict__ status) {
    if (*status) return;
    const int r = blockIdx.y;
    if (r == c) return;
    const double f = fcol[r];
    if (f == 0.0) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    M[(long long)r * N + k] -= f * M[(long long)c * N + k];
    Inv[(long long)r * N + k] -= f * Inv[(long long)c * N + k];
}

void launch_gauss_jordan(double* A, double* Inv, int N, double* fcol, int* status, hipStream_t st) {
    const long long nn = (long long)N * N;
    hipLaunchKernelGGL(k_gj_identity, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, Inv, N, status);
    for (int c = 0; c < N; ++c) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, st, A, Inv, N, c, fcol, status);
        hipLaunchKernelGGL(k_gj_eliminate, dim3((N + 255) / 256, N), dim3(256), 0, st, A, Inv, N, c, fcol, status);
    }
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

// 1/K = exp(-theta) per triangle from the log-permeability theta = ln K
__global__ void k_kinv_from_logK(const double* __restrict__ th, double* __restrict__ kinv, Layout L) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= L.n || j >= L.n) return;
    const long long c = (long long)j * L.n + i;
    const long long nn = (long long)L.n * L.n;
    kinv[slot_index(L, i, j)] = exp(-th[c]);
    kinv[L.plane + slot_index(L, i, j)] = exp(-th[nn + c]);
}

void launch_kinv_from_logK(const double* theta_tri, double* kinv, const Layout& L, hipStream_t st) {
    launch_fill(kinv, 2 * L.plane, 0.0, st);
    dim3 blk(64, 4), grd((L.n + 63) / 64, (L.n + 3) / 4);
    hipLaunchKernelGGL(k_kinv_from_logK, grd, blk, 0, st, theta_tri, kinv, L);
}

// *bad = 1 when a value is unusable: mode 0 (permeability K) unless K > 0 with 1/K finite
// and non-zero; mode 1 (theta = ln K) unless exp(-theta) is finite and non-zero.  Every
// thread that finds one stores the same value.
__global__ void k_check_field(const double* __restrict__ v, long long n, int mode, int* __restrict__ bad) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    bool ok = true;
    for (; e < n; e += stride) {
        const double a = v[e];
        if (mode == 0) {
            const double r = 1.0 / a;
            ok = ok && (a > 0.0) && isfinite(a) && isfinite(r) && r > 0.0;
        } else {
            ok = ok && isfinite(a) && a > -700.0 && a < 700.0;
        }
    }
    if (!ok) *bad = 1;
}

void launch_check_field(const double* v, long long n, int mode, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, st, bad, 1LL, 0);
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_check_field, dim3(std::max(blocks, 1)), dim3(256), 0, st, v, n, mode, bad);
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
