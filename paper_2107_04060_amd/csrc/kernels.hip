// Device kernels of the RQ Biot multigrid for gfx950 (CDNA4, 64-wide wavefronts).
//
// Paper passages: operator -- Sec. 2.1 (block_form), 2.3 (block_form_rq), Appendix A;
// additive Vanka -- Sec. 3.2.1; transfers -- Sec. 3 (eq. block_interp), 3.1; coarse direct
// solve and FGMRES -- Sec. 5.1.
#include "kernels.h"

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
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_apply(const T* __restrict__ x, const T* __restrict__ b,
                                               T* __restrict__ y, const T* __restrict__ kinv, Layout L,
                                               const StencilEntry* __restrict__ st,
                                               const int* __restrict__ st_off) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const long long s = slot_index(L, i, j);
    for (int t = 0; t < NTYPES; ++t) {
        const bool f = dof_free(t, i, j, L.n);
        T acc = 0;
        if (f) {
            const int e0 = st_off[t], e1 = st_off[t + 1];
            for (int e = e0; e < e1; ++e) {
                const StencilEntry E = st[e];
                T c = (T)E.coef;
                if (E.ktri >= 0) c *= kinv[E.ktri * L.plane + s + (long long)E.kdj * L.pitch + E.kdi];
                acc += c * x[E.in_t * L.plane + s + (long long)E.dj * L.pitch + E.di];
            }
        }
        const long long o = t * L.plane + s;
        y[o] = f ? (MODE ? b[o] - acc : acc) : (T)0;
    }
}

template <typename T>
void launch_apply(const LevelView<T>& lv, const T* x, const T* b, T* y, int mode, hipStream_t st) {
    dim3 blk(64, 4);
    dim3 grd((lv.L.n + 1 + 63) / 64, (lv.L.n + 1 + 3) / 4);
    if (mode)
        hipLaunchKernelGGL((k_apply<T, 1>), grd, blk, 0, st, x, b, y, lv.kinv, lv.L, lv.st, lv.st_off);
    else
        hipLaunchKernelGGL((k_apply<T, 0>), grd, blk, 0, st, x, b, y, lv.kinv, lv.L, lv.st, lv.st_off);
}
template void launch_apply<double>(const LevelView<double>&, const double*, const double*, double*, int,
                                   hipStream_t);
template void launch_apply<float>(const LevelView<float>&, const float*, const float*, float*, int, hipStream_t);

// =========================================================================================
// additive Vanka (Sec. 3.2.1)
// =========================================================================================
// Patch solve of one vertex patch by block elimination onto the six pressures:
//   [[A, 0, Bh^T], [0, W, Q^T], [Bh, Q, -C]] (xu, xw, xp) = (ru, rw, rp)
//   S xp = Bh A^-1 ru + Q W^-1 rw - rp,  S = C + Bh A^-1 Bh^T + Q W^-1 Q^T  (SPD),
// with the pressure constant on the star (an exact eigenvector of S with eigenvalue
// (1/M)|T|, since the patch velocities see no net flux of it) solved for in closed form
// and removed from S by a rank-one shift before the Cholesky factorization.
template <typename T>
__device__ inline bool chol6(T A[6][6]) {
#pragma unroll
    for (int jj = 0; jj < 6; ++jj) {
        T d = A[jj][jj];
#pragma unroll
        for (int k = 0; k < jj; ++k) d -= A[jj][k] * A[jj][k];
        if (!(d > (T)0)) return false;
        d = sqrt(d);
        A[jj][jj] = d;
        const T inv = (T)1 / d;
#pragma unroll
        for (int ii = jj + 1; ii < 6; ++ii) {
            T s = A[ii][jj];
#pragma unroll
            for (int k = 0; k < jj; ++k) s -= A[ii][k] * A[jj][k];
            A[ii][jj] = s * inv;
        }
    }
    return true;
}

template <typename T>
__device__ inline void cholsolve6(const T Lm[6][6], T v[6]) {
#pragma unroll
    for (int ii = 0; ii < 6; ++ii) {
        T s = v[ii];
#pragma unroll
        for (int k = 0; k < ii; ++k) s -= Lm[ii][k] * v[k];
        v[ii] = s / Lm[ii][ii];
    }
#pragma unroll
    for (int ii = 5; ii >= 0; --ii) {
        T s = v[ii];
#pragma unroll
        for (int k = ii + 1; k < 6; ++k) s -= Lm[k][ii] * v[k];
        v[ii] = s / Lm[ii][ii];
    }
}

template <typename T>
__device__ void patch_solve(const T rr[PATCH], const DevPatchClass<T>& pc, const T kv[6],
                            const T* __restrict__ wblk, T out[PATCH]) {
    int pres[PATCH];
#pragma unroll
    for (int s = 0; s < PATCH; ++s) pres[s] = pc.present[s];
    // y_u = A^-1 r_u
    T yu[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        T s = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) s += pc.Ainv[a][b] * rr[b];
        yu[a] = s;
    }
    // W (RT0 mass on the six star edges): star triangle k holds the edge pair star_wpair(k, 0..1)
    T W[6][6];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b < 6; ++b) W[a][b] = 0;
#pragma unroll
    for (int kq = 0; kq < 6; ++kq)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int a = star_wpair(kq, p), b = star_wpair(kq, q);
                if (pres[8 + a] && pres[8 + b]) W[a][b] += wblk[(kq * 2 + p) * 2 + q] * kv[kq];
            }
#pragma unroll
    for (int a = 0; a < 6; ++a)
        if (!pres[8 + a]) W[a][a] = 1;
    chol6(W);
    T yw[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) yw[a] = rr[8 + a];
    cholsolve6(W, yw);
    // Z = W^-1 Q^T  (column q = W^-1 Q[q][:]^T)
    T Z[6][6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        T v[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) v[a] = pc.Q[q][a];
        cholsolve6(W, v);
#pragma unroll
        for (int a = 0; a < 6; ++a) Z[a][q] = v[a];
    }
    // S = C + G + Q Z ; rhs = H^T r_u + Q y_w - r_p
    T S[6][6], rhs[6];
    int k = 0;
    T sum_rp = 0, csum = 0, tr = 0;
#pragma unroll
    for (int q1 = 0; q1 < 6; ++q1) {
#pragma unroll
        for (int q2 = 0; q2 < 6; ++q2) {
            T s = pc.G[q1][q2];
#pragma unroll
            for (int a = 0; a < 6; ++a) s += pc.Q[q1][a] * Z[a][q2];
            S[q1][q2] = s;
        }
        S[q1][q1] += pc.c[q1];
        T s = -rr[14 + q1];
#pragma unroll
        for (int a = 0; a < 8; ++a) s += pc.H[a][q1] * rr[a];
#pragma unroll
        for (int a = 0; a < 6; ++a) s += pc.Q[q1][a] * yw[a];
        rhs[q1] = s;
        if (pres[14 + q1]) {
            ++k;
            sum_rp += rr[14 + q1];
            csum += pc.c[q1];
            tr += S[q1][q1];
        }
    }
    // star-mean pressure: x_p = x_perp + gamma 1 with gamma = (1^T rhs) / (k c0) = -sum(r_p) / sum(c)
    const T gamma = -sum_rp / csum;
    T mrhs = 0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (pres[14 + q]) mrhs += rhs[q];
    mrhs /= (T)k;
    const T beta = tr / (T)(k * k);
#pragma unroll
    for (int q1 = 0; q1 < 6; ++q1) {
#pragma unroll
        for (int q2 = 0; q2 < 6; ++q2) {
            if (pres[14 + q1] && pres[14 + q2])
                S[q1][q2] += beta;
            else
                S[q1][q2] = (q1 == q2) ? (T)1 : (T)0;
        }
        rhs[q1] = pres[14 + q1] ? rhs[q1] - mrhs : (T)0;
    }
    chol6(S);
    cholsolve6(S, rhs);
    T xp[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) xp[q] = pres[14 + q] ? rhs[q] + gamma : (T)0;
    // back substitution
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        T s = yu[a];
#pragma unroll
        for (int q = 0; q < 6; ++q) s -= pc.H[a][q] * xp[q];
        out[a] = pres[a] ? s : (T)0;
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        T s = yw[a];
#pragma unroll
        for (int q = 0; q < 6; ++q) s -= Z[a][q] * xp[q];
        out[8 + a] = pres[8 + a] ? s : (T)0;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) out[14 + q] = xp[q];
}

constexpr int VT = 16;       // patches per tile side (threads)
constexpr int VO = VT - 1;   // owned slots per tile side

__device__ inline double vanka_weight(int t, int i, int j, int n) {
    if (t <= T_UY) return 1.0;
    if (t <= T_WD) return 0.5;
    if (t == T_PL) return (i == 0 && j == 0) ? 0.5 : 1.0 / 3.0;
    return (i == n - 1 && j == n - 1) ? 0.5 : 1.0 / 3.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_vanka(const T* __restrict__ r, T* __restrict__ x,
                                               const T* __restrict__ kinv, Layout L,
                                               const DevPatchClass<T>* __restrict__ cls,
                                               const T* __restrict__ wblk, T omega, int x_is_zero) {
    __shared__ T sr[NTYPES][VT + 1][VT + 1];
    __shared__ T sc[PATCH][VT][VT];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * VT + tx;
    const int i0 = blockIdx.x * VO, j0 = blockIdx.y * VO;
    const int n = L.n;
    // stage the residual of slots (i0-1 .. i0+VT-1) x (j0-1 .. j0+VT-1)
    constexpr int TS = (VT + 1) * (VT + 1);
    for (int q = tid; q < NTYPES * TS; q += VT * VT) {
        const int t = q / TS, rem = q - t * TS, bb = rem / (VT + 1), aa = rem - bb * (VT + 1);
        const int si = i0 - 1 + aa, sj = j0 - 1 + bb;
        T v = 0;
        if (si >= -1 && si <= n + 1 && sj >= -1 && sj <= n + 1) v = r[t * L.plane + slot_index(L, si, sj)];
        sr[t][bb][aa] = v;
    }
    __syncthreads();
    const int vi = i0 + tx, vj = j0 + ty;
    T out[PATCH];
#pragma unroll
    for (int s = 0; s < PATCH; ++s) out[s] = 0;
    if (vi <= n && vj <= n) {
        const int ci = vi == 0 ? 0 : (vi == n ? 2 : 1);
        const int cj = vj == 0 ? 0 : (vj == n ? 2 : 1);
        const DevPatchClass<T>& pc = cls[3 * cj + ci];
        bool keep = false;
#pragma unroll
        for (int s = 0; s < 14; ++s) keep = keep || pc.present[s];
        if (keep) {
            T rr[PATCH];
#pragma unroll
            for (int s = 0; s < PATCH; ++s) {
                int t, di, dj;
                patch_slot(s, t, di, dj);
                rr[s] = sr[t][ty + 1 + dj][tx + 1 + di];
            }
            T kv[6];
#pragma unroll
            for (int kq = 0; kq < 6; ++kq) {
                int ut, di, dj;
                star_tri(kq, ut, di, dj);
                kv[kq] = kinv[ut * L.plane + slot_index(L, vi + di, vj + dj)];
            }
            patch_solve<T>(rr, pc, kv, wblk, out);
        }
    }
#pragma unroll
    for (int s = 0; s < PATCH; ++s) sc[s][ty][tx] = out[s];
    __syncthreads();
    if (tx < VO && ty < VO) {
        const int si = i0 + tx, sj = j0 + ty;
        if (si <= n && sj <= n) {
            T c[NTYPES];
            c[T_UX] = sc[0][ty][tx];
            c[T_UY] = sc[1][ty][tx];
            c[T_BH] = sc[3][ty][tx] + sc[2][ty][tx + 1];
            c[T_BV] = sc[5][ty][tx] + sc[4][ty + 1][tx];
            c[T_BD] = sc[6][ty][tx + 1] + sc[7][ty + 1][tx];
            c[T_WH] = sc[9][ty][tx] + sc[8][ty][tx + 1];
            c[T_WV] = sc[11][ty][tx] + sc[10][ty + 1][tx];
            c[T_WD] = sc[12][ty][tx + 1] + sc[13][ty + 1][tx];
            c[T_PL] = sc[14][ty][tx] + sc[15][ty][tx + 1] + sc[16][ty + 1][tx];
            c[T_PU] = sc[17][ty + 1][tx + 1] + sc[18][ty][tx + 1] + sc[19][ty + 1][tx];
            const long long s0 = slot_index(L, si, sj);
#pragma unroll
            for (int t = 0; t < NTYPES; ++t) {
                if (!dof_free(t, si, sj, n)) continue;
                const long long o = t * L.plane + s0;
                const T w = (T)vanka_weight(t, si, sj, n);
                const T old = x_is_zero ? (T)0 : x[o];
                x[o] = old + omega * w * c[t];
            }
        }
    }
}

template <typename T>
void launch_vanka(const LevelView<T>& lv, const T* r, T* x, T omega, int x_is_zero, hipStream_t st) {
    dim3 blk(VT, VT);
    dim3 grd((lv.L.n + 1 + VO - 1) / VO, (lv.L.n + 1 + VO - 1) / VO);
    hipLaunchKernelGGL(k_vanka<T>, grd, blk, 0, st, r, x, lv.kinv, lv.L, lv.cls, lv.wblk, omega, x_is_zero);
}
template void launch_vanka<double>(const LevelView<double>&, const double*, double*, double, int, hipStream_t);
template void launch_vanka<float>(const LevelView<float>&, const float*, float*, float, int, hipStream_t);

// =========================================================================================
// grid transfers (Sec. 3, 3.1): gather forms of P^T and P
// =========================================================================================
template <typename T>
__global__ void k_restrict(const T* __restrict__ rf, T* __restrict__ rc, Layout Lf, Layout Lc,
                           const RestrictEntry* __restrict__ tab, const int* __restrict__ off) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I > Lc.n || J > Lc.n) return;
    const long long sc = slot_index(Lc, I, J);
    for (int t = 0; t < NTYPES; ++t) {
        T acc = 0;
        const bool f = dof_free(t, I, J, Lc.n);
        if (f) {
            for (int e = off[t]; e < off[t + 1]; ++e) {
                const RestrictEntry E = tab[e];
                const int fi = 2 * I + E.di, fj = 2 * J + E.dj;
                if (fi < -1 || fi > Lf.n + 1 || fj < -1 || fj > Lf.n + 1) continue;
                acc += (T)E.w * rf[E.t_f * Lf.plane + slot_index(Lf, fi, fj)];
            }
        }
        rc[t * Lc.plane + sc] = f ? acc : (T)0;
    }
}

template <typename T>
void launch_restrict(const Layout& Lf, const Layout& Lc, const T* rf, T* rc, const RestrictEntry* tab,
                     const int* off, hipStream_t st) {
    dim3 blk(64, 4);
    dim3 grd((Lc.n + 1 + 63) / 64, (Lc.n + 1 + 3) / 4);
    hipLaunchKernelGGL(k_restrict<T>, grd, blk, 0, st, rf, rc, Lf, Lc, tab, off);
}
template void launch_restrict<double>(const Layout&, const Layout&, const double*, double*, const RestrictEntry*,
                                      const int*, hipStream_t);
template void launch_restrict<float>(const Layout&, const Layout&, const float*, float*, const RestrictEntry*,
                                     const int*, hipStream_t);

// off: 41 offsets, group g = (t_f * 2 + pi) * 2 + pj
template <typename T>
__global__ void k_prolong_add(const T* __restrict__ xc, T* __restrict__ xf, Layout Lf, Layout Lc,
                              const ProlongEntry* __restrict__ tab, const int* __restrict__ off) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I > Lc.n || J > Lc.n) return;
    for (int pj = 0; pj < 2; ++pj)
        for (int pi = 0; pi < 2; ++pi) {
            const int fi = 2 * I + pi, fj = 2 * J + pj;
            if (fi > Lf.n || fj > Lf.n) continue;
            const long long sf = slot_index(Lf, fi, fj);
            for (int t = 0; t < NTYPES; ++t) {
                if (!dof_free(t, fi, fj, Lf.n)) continue;
                const int g = (t * 2 + pi) * 2 + pj;
                T acc = 0;
                for (int e = off[g]; e < off[g + 1]; ++e) {
                    const ProlongEntry E = tab[e];
                    const int ci = I + E.dI, cj = J + E.dJ;
                    if (ci < -1 || ci > Lc.n + 1 || cj < -1 || cj > Lc.n + 1) continue;
                    acc += (T)E.w * xc[E.t_c * Lc.plane + slot_index(Lc, ci, cj)];
                }
                xf[t * Lf.plane + sf] += acc;
            }
        }
}

template <typename T>
void launch_prolong_add(const Layout& Lf, const Layout& Lc, const T* xc, T* xf, const ProlongEntry* tab,
                        const int* off, hipStream_t st) {
    dim3 blk(64, 4);
    dim3 grd((Lc.n + 1 + 63) / 64, (Lc.n + 1 + 3) / 4);
    hipLaunchKernelGGL(k_prolong_add<T>, grd, blk, 0, st, xc, xf, Lf, Lc, tab, off);
}
template void launch_prolong_add<double>(const Layout&, const Layout&, const double*, double*, const ProlongEntry*,
                                         const int*, hipStream_t);
template void launch_prolong_add<float>(const Layout&, const Layout&, const float*, float*, const ProlongEntry*,
                                        const int*, hipStream_t);

// =========================================================================================
// coarsest level: dense inverse applied by one workgroup (Sec. 5.1 direct solve)
// =========================================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(const double* __restrict__ Ainv, int N,
                                                      const int* __restrict__ idx, const T* __restrict__ b,
                                                      T* __restrict__ x) {
    extern __shared__ double bb[];
    for (int k = threadIdx.x; k < N; k += blockDim.x) bb[k] = (double)b[idx[k]];
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        double s = 0;
        const double* row = Ainv + (long long)k * N;
        for (int l = 0; l < N; ++l) s += row[l] * bb[l];
        x[idx[k]] = (T)s;
    }
}

template <typename T>
void launch_coarse_solve(const double* Ainv, int N, const int* idx, const T* b, T* x, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse_solve<T>, dim3(1), dim3(256), N * sizeof(double), st, Ainv, N, idx, b, x);
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
// Krylov BLAS-1 (FP64, deterministic two-stage reductions)
// =========================================================================================
__global__ __launch_bounds__(256) void k_multidot(const double* __restrict__ V, long long ldv, int nv,
                                                  const double* __restrict__ w, long long n,
                                                  double* __restrict__ partial) {
    __shared__ double red[4][256];
    const long long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    for (int v0 = 0; v0 < nv; v0 += 4) {
        double acc[4] = {0, 0, 0, 0};
        for (long long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
            const double we = w[e];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (v0 + q < nv) acc[q] += V[(long long)(v0 + q) * ldv + e] * we;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = acc[q];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s)
#pragma unroll
                for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x < 4 && v0 + (int)threadIdx.x < nv)
            partial[(long long)blockIdx.x * nv + v0 + threadIdx.x] = red[threadIdx.x][0];
        __syncthreads();
    }
}

void launch_multidot(const double* V, long long ldv, int nv, const double* w, long long n, double* partial,
                     int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_multidot, dim3(nblk), dim3(256), 0, st, V, ldv, nv, w, n, partial);
}

__global__ void k_reduce_partials(const double* __restrict__ partial, int nblk, int nv, double* __restrict__ out,
                                  int accumulate) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    double s = 0;
    for (int b = 0; b < nblk; ++b) s += partial[(long long)b * nv + v];
    out[v] = accumulate ? out[v] + s : s;
}

void launch_reduce_partials(const double* partial, int nblk, int nv, double* out, int accumulate,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partials, dim3((nv + 63) / 64), dim3(64), 0, st, partial, nblk, nv, out,
                       accumulate);
}

__global__ void k_update(double* __restrict__ w, const double* __restrict__ V, long long ldv, int nv,
                         const double* __restrict__ h, long long n) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < n; e += stride) {
        double s = w[e];
        for (int q = 0; q < nv; ++q) s -= h[q] * V[(long long)q * ldv + e];
        w[e] = s;
    }
}

void launch_update(double* w, const double* V, long long ldv, int nv, const double* h, long long n,
                   hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_update, dim3(blocks), dim3(256), 0, st, w, V, ldv, nv, h, n);
}

__global__ void k_scale_inv_sqrt(double* __restrict__ dst, const double* __restrict__ src, long long n,
                                 const double* __restrict__ norm2) {
    const double s = 1.0 / sqrt(*norm2);
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < n; e += stride) dst[e] = src[e] * s;
}

void launch_scale_inv_sqrt(double* dst, const double* src, long long n, const double* norm2, hipStream_t st) {
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(blocks), dim3(256), 0, st, dst, src, n, norm2);
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
