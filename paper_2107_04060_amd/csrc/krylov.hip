// FGMRES vector kernels (Sec. 5.1): classical Gram-Schmidt passes with deterministic two-stage
// reductions, normalization, scaling and the solution update.
#include "kernels.h"
#include "tile.h"

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include <hip/hip_runtime.h>

namespace biot {

// =========================================================================================
// Krylov BLAS-1 (FP64, deterministic reductions)
// =========================================================================================
// ---- classical Gram-Schmidt pass: dots, update with norm, deterministic reductions ----------------
// The partial sums of each block go to partial[q * np + b] (np blocks); a second kernel adds them
// in a fixed order.  Kernels given run_if return at once when *run_if == 0.
constexpr int DOT_BLOCKS = RED_BLOCKS;     // dot-product blocks (contiguous chunks)
constexpr int UPD_BLOCKS = 4 * RED_BLOCKS; // update blocks (grid stride)


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

// Single pass over V_q (q < nv <= NVB <= GS_FUSED) and w: partial sums of V_q . w (slots
// 0..nv-1) and w . w (slot nv).  UPDATE: first w -= sum_q h[q] V_q, the sums then taken on the new
// w (the dot products of the next Gram-Schmidt pass, taken while V is read for this one).
// Contiguous chunks per block; every element's V_q are loaded at once and stay in registers,
// sized by the bucket NVB (8, 16 or 32) so that short bases keep more waves resident.  VEC = 2:
// each lane moves two consecutive elements per 16-byte load (n even, vectors 16-byte aligned).
// blocks of the single-pass kernels: 512 contiguous chunks up to 4 M elements (fastest there),
// 1024 above (more 16-byte loads in flight on the 2048^2 mesh's vectors)
static int fused_blocks(long long n) { return n >= (1LL << 22) ? 1024 : 512; }
static_assert(1024 <= RED_BLOCKS, "the partial-sum buffer holds RED_BLOCKS sums per slot");
template <bool UPDATE, int NVB, int VEC>
__global__ __launch_bounds__(256) void k_gs_fused(double* __restrict__ w, const double* __restrict__ V,
                                                  long long ldv, int nv, const double* __restrict__ h,
                                                  long long n, double* __restrict__ partial,
                                                  const double* run_if) {
    static_assert(NVB <= GS_FUSED && (VEC == 1 || VEC == 2), "fused Gram-Schmidt bucket");
    using vec_t = std::conditional_t<VEC == 2, double2, double>;
    if (run_if && *run_if == 0.0) return;
    __shared__ double red[4][NVB + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long ng = n / VEC;                               // element groups (n % VEC == 0)
    const long long chunk = (ng + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(ng, lo + chunk);
    double hq[NVB], acc[NVB + 1];
#pragma unroll
    for (int q = 0; q < NVB; ++q) hq[q] = (UPDATE && q < nv) ? h[q] : 0.0;
#pragma unroll
    for (int q = 0; q <= NVB; ++q) acc[q] = 0;
    const vec_t* Vv = reinterpret_cast<const vec_t*>(V);
    vec_t* wv = reinterpret_cast<vec_t*>(w);
    const long long ldg = ldv / VEC;
    for (long long g = lo + threadIdx.x; g < hi; g += blockDim.x) {
        if constexpr (VEC == 2) {
            double2 v[NVB];
#pragma unroll
            for (int q = 0; q < NVB; ++q) v[q] = q < nv ? Vv[(long long)q * ldg + g] : double2{0.0, 0.0};
            double2 sv = wv[g];
            if constexpr (UPDATE) {
#pragma unroll
                for (int q = 0; q < NVB; ++q) {
                    sv.x -= hq[q] * v[q].x;
                    sv.y -= hq[q] * v[q].y;
                }
                wv[g] = sv;
            }
#pragma unroll
            for (int q = 0; q < NVB; ++q) {
                acc[q] += v[q].x * sv.x;
                acc[q] += v[q].y * sv.y;
            }
            acc[NVB] += sv.x * sv.x;
            acc[NVB] += sv.y * sv.y;
        } else {
            double v[NVB];
#pragma unroll
            for (int q = 0; q < NVB; ++q) v[q] = q < nv ? Vv[(long long)q * ldg + g] : 0.0;
            double sv = wv[g];
            if constexpr (UPDATE) {
#pragma unroll
                for (int q = 0; q < NVB; ++q) sv -= hq[q] * v[q];
                wv[g] = sv;
            }
#pragma unroll
            for (int q = 0; q < NVB; ++q) acc[q] += v[q] * sv;
            acc[NVB] += sv * sv;
        }
    }
    // output slots: q < nv the dot products, nv the w . w (accumulated in acc[NVB])
#pragma unroll
    for (int q = 0; q <= NVB; ++q) {
        if (q < nv || q == NVB) {
            const double t = wave_sum(acc[q]);
            if (lane == 0) red[wave][q] = t;
        }
    }
    __syncthreads();
    const int q = threadIdx.x;
    if (q < nv || q == NVB) {
        const double r = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
        partial[(long long)(q == NVB ? nv : q) * gridDim.x + blockIdx.x] = r;
    }
}

// launch k_gs_fused on the smallest register bucket that holds nv vectors
template <bool UPDATE>
static void launch_gs_fused(double* w, const double* V, long long ldv, int nv, const double* h, long long n,
                            double* partial, const double* run_if, hipStream_t st) {
    const bool v2 = n % 2 == 0 && ldv % 2 == 0 && reinterpret_cast<uintptr_t>(V) % 16 == 0 &&
                    reinterpret_cast<uintptr_t>(w) % 16 == 0;
    const dim3 grd(fused_blocks(n)), blk(256);
#define BIOT_GS_FUSED(NVB)                                                                                      \
    do {                                                                                                      \
        if (v2)                                                                                               \
            hipLaunchKernelGGL((k_gs_fused<UPDATE, NVB, 2>), grd, blk, 0, st, w, V, ldv, nv, h, n, partial,      \
                               run_if);                                                                       \
        else                                                                                                  \
            hipLaunchKernelGGL((k_gs_fused<UPDATE, NVB, 1>), grd, blk, 0, st, w, V, ldv, nv, h, n, partial,      \
                               run_if);                                                                       \
    } while (0)
    if (nv <= 8)
        BIOT_GS_FUSED(8);
    else if (nv <= 16)
        BIOT_GS_FUSED(16);
    else
        BIOT_GS_FUSED(32);
#undef BIOT_GS_FUSED
}

// out[q] = sum_b partial[q * np + b], one block per q (fixed order); host: optional mirror.
// flag (optional): set by the block of q == flag_q to 1 when out[flag_q] < eta2 * prev (the
// Daniel-Gragg-Kaufman-Stewart test for a second orthogonalization pass on squared norms,
// eta2 = eta^2, eta = 1/sqrt(2) by default), and mirrored to *host_flag when given.
__global__ __launch_bounds__(256) void k_gs_reduce(const double* __restrict__ partial, int np,
                                                   double* __restrict__ out, double* __restrict__ host,
                                                   const double* __restrict__ prev, double* __restrict__ flag,
                                                   double* __restrict__ host_flag, int flag_q,
                                                   const double* run_if, double eta2) {
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
        if (flag && q == flag_q) {
            const double f = (r < eta2 * (*prev)) ? 1.0 : 0.0;
            *flag = f;
            if (host_flag) *host_flag = f;
        }
    }
}

void launch_gs_dots(const double* V, long long ldv, int nv, const double* w, long long n, double* partial,
                    double* out, double* host, const double* run_if, hipStream_t st) {
    // one pass over all vectors up to GS_FUSED of them, else groups of GSV per pass
    const int np = nv <= GS_FUSED ? fused_blocks(n) : DOT_BLOCKS;
    if (nv <= GS_FUSED)
        launch_gs_fused<false>(const_cast<double*>(w), V, ldv, nv, nullptr, n, partial, run_if, st);
    else
        hipLaunchKernelGGL(k_gs_dots, dim3(np), dim3(256), 0, st, V, ldv, nv, w, n, partial, run_if);
    hipLaunchKernelGGL(k_gs_reduce, dim3(nv + 1), dim3(256), 0, st, partial, np, out, host, nullptr,
                       nullptr, nullptr, 0, run_if, 0.0);
}

void launch_gs_update(double* w, const double* V, long long ldv, int nv, const double* h, long long n,
                      double* partial, double* norm2, const double* prev, double* flag, double* host,
                      const double* run_if, hipStream_t st, double eta2) {
    hipLaunchKernelGGL(k_gs_update, dim3(UPD_BLOCKS), dim3(256), 0, st, w, V, ldv, nv, h, n, partial, run_if);
    hipLaunchKernelGGL(k_gs_reduce, dim3(1), dim3(256), 0, st, partial, UPD_BLOCKS, norm2, host, prev, flag,
                       host ? host + 1 : nullptr, 0, run_if, eta2);
}

void launch_gs_update_dots(double* w, const double* V, long long ldv, int nv, const double* h, long long n,
                           double* partial, double* out, double* host, const double* prev, double* flag,
                           double* host_flag, hipStream_t st, double eta2) {
    if (nv < 1 || nv > GS_FUSED) throw ArgError{"fused Gram-Schmidt pass: 1 <= nv <= GS_FUSED"};
    launch_gs_fused<true>(w, V, ldv, nv, h, n, partial, nullptr, st);
    hipLaunchKernelGGL(k_gs_reduce, dim3(nv + 1), dim3(256), 0, st, partial, fused_blocks(n), out, host, prev, flag,
                       host_flag, nv, nullptr, eta2);
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

}  // namespace biot
