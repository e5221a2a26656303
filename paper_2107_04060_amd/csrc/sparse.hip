// Kernels of the general-boundary path (sparse.h): CSR products, on-device assembly of the
// operator values from per-triangle 1/K, and the additive Vanka step on explicit patch
// inverses.  Paper: Sec. 2.1 (K enters tau M_w(K) only), Sec. 3 (R = P^T), Sec. 3.2.1 (additive
// Vanka: x <- x + omega sum_l V_l^T D_l A_l^{-1} V_l (b - A x)), Sec. 5 (Terzaghi: the Vanka
// blocks shifted by a small weight on the diagonal when M = infinity).
//
// These levels are small (the path serves meshes up to 256 x 256) and their launches latency
// bound: a CSR row is spread over LPR lanes (a few entries each, then a butterfly sum), a
// patch entry's 20 loads are issued together (full unroll), so that no thread walks a long
// chain of dependent loads.
#include "sparse.h"

namespace biot {

namespace {

constexpr int TPB = 256;
constexpr int LPR = 8;   // lanes per CSR row (consecutive lanes of one wave)

inline unsigned blocks(long long n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

// every lane of a wave takes part in the butterfly, rows past the end with zero sums
__global__ __launch_bounds__(TPB) void k_csr_mv(int rows, const int* __restrict__ ptr, const int* __restrict__ col,
                                                const double* __restrict__ val, const double* __restrict__ x,
                                                const double* z, double* y, double a, double c) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long r = t / LPR;
    const int lane = (int)(t % LPR);
    double s = 0.0;
    if (r < rows && x)
        for (int q = ptr[r] + lane; q < ptr[r + 1]; q += LPR) s += val[q] * x[col[q]];
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR);
    if (r < rows && lane == 0) y[r] = (z ? c * z[r] : 0.0) + a * s;
}

__global__ __launch_bounds__(TPB) void k_csr_assemble(int nnz, const double* __restrict__ val0,
                                                      const int* __restrict__ kptr, const int* __restrict__ ktri,
                                                      const double* __restrict__ kcoef,
                                                      const double* __restrict__ kinv, double* __restrict__ val) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    double v = val0[e];
    for (int q = kptr[e]; q < kptr[e + 1]; ++q) v += kcoef[q] * kinv[ktri[q]];
    val[e] = v;
}

__global__ __launch_bounds__(TPB) void k_kinv_flat(long long ntri, const double* __restrict__ K, double Ks, int mode,
                                                   double* __restrict__ kinv) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntri) return;
    kinv[t] = mode == 1 ? exp(-K[t]) : 1.0 / (K ? K[t] : Ks);
}

// coarse L(I, J) = {(2I, 2J), (2I+2, 2J), (2I, 2J+2)} in fine units: children L(2I, 2J),
// L(2I+1, 2J), L(2I, 2J+1) and the middle U(2I, 2J); coarse U(I, J): U(2I+1, 2J), U(2I+1, 2J+1),
// U(2I, 2J+1) and the middle L(2I+1, 2J+1)
__global__ __launch_bounds__(TPB) void k_kinv_coarsen_flat(int nc, const double* __restrict__ kf,
                                                           double* __restrict__ kc) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int nn = nc * nc;
    if (q >= 2 * nn) return;
    const int upper = q >= nn, c = q - upper * nn, I = c % nc, J = c / nc;
    const int nf = 2 * nc, mf = nf * nf;
    auto L = [&](int i, int j) { return kf[j * nf + i]; };
    auto U = [&](int i, int j) { return kf[mf + j * nf + i]; };
    const double s = upper ? (U(2 * I + 1, 2 * J) + U(2 * I + 1, 2 * J + 1)) + (U(2 * I, 2 * J + 1) + L(2 * I + 1, 2 * J + 1))
                           : (L(2 * I, 2 * J) + L(2 * I + 1, 2 * J)) + (L(2 * I, 2 * J + 1) + U(2 * I, 2 * J));
    kc[q] = 0.25 * s;
}

// One wave per patch: the 20 x 20 shifted patch matrix (identity on absent slots) next to the
// identity in LDS, Gauss-Jordan with partial pivoting over the rows, the inverse written
// column-major (inv[p][b * 20 + a] = A_p^{-1}[a][b]) so that the apply reads it coalesced.
constexpr int PW = 2 * PATCH;
__global__ __launch_bounds__(64) void k_patch_inverse(int np, const int* __restrict__ slots,
                                                      const int* __restrict__ ptr, const int* __restrict__ col,
                                                      const double* __restrict__ val, double shift,
                                                      double* __restrict__ inv, int* __restrict__ status) {
    __shared__ double M[PATCH][PW + 1];
    __shared__ int sl[PATCH];
    __shared__ int piv;
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    if (p >= np) return;
    if (lane < PATCH) sl[lane] = slots[(long long)p * PATCH + lane];
    __syncthreads();
    for (int e = lane; e < PATCH * PW; e += 64) {
        const int a = e / PW, b = e % PW;
        double v = 0.0;
        if (b >= PATCH) {
            v = (b - PATCH == a) ? 1.0 : 0.0;
        } else if (sl[a] < 0 || sl[b] < 0) {
            v = (a == b) ? 1.0 : 0.0;
        } else {
            // entry (sl[a], sl[b]) of the CSR row: binary search over the sorted columns
            int lo = ptr[sl[a]], hi = ptr[sl[a] + 1] - 1;
            const int want = sl[b];
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = col[mid];
                if (cm == want) {
                    v = val[mid];
                    break;
                }
                if (cm < want) lo = mid + 1;
                else hi = mid - 1;
            }
            if (a == b) v += (a < 14 ? shift : -shift);
        }
        M[a][b] = v;
    }
    __syncthreads();
    for (int k = 0; k < PATCH; ++k) {
        if (lane == 0) {
            int best = k;
            double bv = fabs(M[k][k]);
            for (int r = k + 1; r < PATCH; ++r)
                if (fabs(M[r][k]) > bv) {
                    bv = fabs(M[r][k]);
                    best = r;
                }
            piv = best;
            if (!(bv > 0.0) || !isfinite(bv)) *status = 1;
        }
        __syncthreads();
        const int r0 = piv;
        if (r0 != k)
            for (int b = lane; b < PW; b += 64) {
                const double t = M[k][b];
                M[k][b] = M[r0][b];
                M[r0][b] = t;
            }
        __syncthreads();
        const double d = M[k][k];
        const double rd = d != 0.0 ? 1.0 / d : 0.0;
        __syncthreads();
        for (int b = lane; b < PW; b += 64) M[k][b] *= rd;
        __syncthreads();
        for (int e = lane; e < PATCH * PW; e += 64) {
            const int r = e / PW, b = e % PW;
            if (r == k) continue;
            const double f = M[r][k];
            if (b != k) M[r][b] -= f * M[k][b];
        }
        __syncthreads();
        // column k of the other rows is zero now (kept out of the loop above so that every
        // thread read the old M[r][k])
        if (lane < PATCH && lane != k) M[lane][k] = 0.0;
        __syncthreads();
    }
    double* out = inv + (long long)p * PATCH * PATCH;
    for (int e = lane; e < PATCH * PATCH; e += 64) {
        const int b = e / PATCH, a = e % PATCH;
        out[e] = M[a][PATCH + b];
    }
}

// The slot indices are loaded first (five 16-byte loads), then every residual entry with an
// unconditional load (absent slots read entry 0 and are selected away): no branch between the
// loads, so the 20 gathers are in flight together instead of one after another.
__global__ __launch_bounds__(TPB) void k_patch_apply(int np, const int* __restrict__ slots,
                                                     const double* __restrict__ inv, const double* __restrict__ r,
                                                     double* __restrict__ y) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)np * PATCH) return;
    const long long p = t / PATCH;
    const int a = (int)(t - p * PATCH);
    const int4* s4 = reinterpret_cast<const int4*>(slots + p * PATCH);   // 80-byte rows: 16-byte aligned
    int q[PATCH];
#pragma unroll
    for (int k = 0; k < PATCH / 4; ++k) {
        const int4 v = s4[k];
        q[4 * k] = v.x;
        q[4 * k + 1] = v.y;
        q[4 * k + 2] = v.z;
        q[4 * k + 3] = v.w;
    }
    const double* A = inv + p * PATCH * PATCH + a;
    double v = 0.0;
#pragma unroll
    for (int b = 0; b < PATCH; ++b) {
        const double rb = r[q[b] >= 0 ? q[b] : 0];
        v += A[b * PATCH] * (q[b] >= 0 ? rb : 0.0);
    }
    y[t] = slots[t] >= 0 ? v : 0.0;
}

// multiplicative colour step: as k_patch_apply for the colour's patches, the correction added
// to the iterate in place (the colour's patches are disjoint: every DoF is written by at most one
// thread)
__global__ __launch_bounds__(TPB) void k_patch_apply_add(int npc, const int* __restrict__ plist,
                                                         const int* __restrict__ slots,
                                                         const double* __restrict__ inv, const double* __restrict__ r,
                                                         double omega, double* __restrict__ x) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)npc * PATCH) return;
    const long long k = t / PATCH;
    const int a = (int)(t - k * PATCH);
    const long long p = plist[k];
    const int4* s4 = reinterpret_cast<const int4*>(slots + p * PATCH);
    int q[PATCH];
#pragma unroll
    for (int m = 0; m < PATCH / 4; ++m) {
        const int4 v = s4[m];
        q[4 * m] = v.x;
        q[4 * m + 1] = v.y;
        q[4 * m + 2] = v.z;
        q[4 * m + 3] = v.w;
    }
    const double* A = inv + p * PATCH * PATCH + a;
    double v = 0.0;
#pragma unroll
    for (int b = 0; b < PATCH; ++b) {
        const double rb = r[q[b] >= 0 ? q[b] : 0];
        v += A[b * PATCH] * (q[b] >= 0 ? rb : 0.0);
    }
    const int d = slots[p * PATCH + a];
    if (d >= 0) x[d] += omega * v;
}

// One fused colour step of multiplicative Vanka, in place: per patch of the colour, the residual
// of its 20 rows (LPR_C lanes per row, butterfly sum), then the explicit inverse applied and the
// correction added to x.  In place is safe: a patch's rows couple only DoFs on the triangles of
// its vertex's star, and no other patch of the colour owns one of those (vertices of one colour
// share no mesh edge, so their stars share no triangle, edge or vertex); every x a block reads
// is therefore either its own patch's, written by the block after its reads, or another
// colour's, not written in this launch.  xzero: the iterate is zero (the residual is b, x is not
// read): the corrections are assigned, and blocks past the colour's patches write the zeros of
// the DoFs no patch of the colour holds (zlist, nz), so that x needs no clearing beforehand.
// The colour's rows are listed per (patch, slot) with their CSR bounds (crow, cbeg, cend), so
// that a lane reaches x in three dependent loads; a phase-2 thread loads its inverse column
// before the barrier.
constexpr int LPR_C = 4;                                  // lanes per row
constexpr int PPB_C = TPB / (PATCH * LPR_C);              // patches per block (3)
__global__ __launch_bounds__(TPB) void k_colour_step(int npc, const int* __restrict__ plist,
                                                     const int* __restrict__ crow, const int* __restrict__ cbeg,
                                                     const int* __restrict__ cend, const double* __restrict__ inv,
                                                     const int* __restrict__ col, const double* __restrict__ val,
                                                     const double* __restrict__ b, double* x, double omega,
                                                     int xzero, const int* __restrict__ zlist, int nz) {
    __shared__ double rsh[PPB_C][PATCH];
    const int t = threadIdx.x;
    const int npb = (npc + PPB_C - 1) / PPB_C;
    if ((int)blockIdx.x >= npb) {
        // zero-start: the DoFs outside the colour's patches
        const long long z = (long long)(blockIdx.x - npb) * blockDim.x + t;
        if (z < nz) x[zlist[z]] = 0.0;
        return;
    }
    const int k0 = blockIdx.x * PPB_C;
    // phase 2's inverse column, loaded first (independent of phase 1)
    const bool p2 = t < PPB_C * PATCH && k0 + t / PATCH < npc;
    double ac[PATCH];
    if (p2) {
        const long long p = plist[k0 + t / PATCH];
        const double* A = inv + p * PATCH * PATCH + t % PATCH;
#pragma unroll
        for (int bb = 0; bb < PATCH; ++bb) ac[bb] = A[bb * PATCH];
    }
    // phase 1: residual rows
    {
        const int kl = t / (PATCH * LPR_C), a = (t / LPR_C) % PATCH, sub = t % LPR_C;
        const long long e = (long long)(k0 + kl) * PATCH + a;
        const bool live = kl < PPB_C && k0 + kl < npc;
        const int d = live ? crow[e] : -1;
        double s = 0.0;
        if (d >= 0 && !xzero) {
            const int hi = cend[e];
            for (int q = cbeg[e] + sub; q < hi; q += LPR_C) s += val[q] * x[col[q]];
        }
#pragma unroll
        for (int o = LPR_C / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR_C);
        if (kl < PPB_C && sub == 0) rsh[kl][a] = d >= 0 ? b[d] - s : 0.0;
    }
    __syncthreads();
    // phase 2: correction of slot a of patch kl
    if (p2) {
        const int kl = t / PATCH, a = t % PATCH;
        double v = 0.0;
#pragma unroll
        for (int bb = 0; bb < PATCH; ++bb) v += ac[bb] * rsh[kl][bb];
        const int d = crow[(long long)(k0 + kl) * PATCH + a];
        if (d >= 0) x[d] = (xzero ? 0.0 : x[d]) + omega * v;
    }
}

__global__ __launch_bounds__(TPB) void k_kinv_unpad(Layout L, const double* __restrict__ kp, double* __restrict__ kf) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nn = (long long)L.n * L.n;
    if (q >= 2 * nn) return;
    const int u = q >= nn;
    const long long c = q - u * nn;
    const int i = (int)(c % L.n), j = (int)(c / L.n);
    kf[q] = kp[u * L.plane + slot_index(L, i, j)];
}

__global__ __launch_bounds__(TPB) void k_patch_gather(int N, const int* __restrict__ dptr,
                                                      const int* __restrict__ dlist, const double* __restrict__ y,
                                                      const double* __restrict__ wgt, double omega, const double* x,
                                                      double* xout) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= N) return;
    double s = 0.0;
    for (int q = dptr[d]; q < dptr[d + 1]; ++q) s += y[dlist[q]];
    xout[d] = (x ? x[d] : 0.0) + omega * wgt[d] * s;
}

__global__ __launch_bounds__(TPB) void k_csr_to_dense(int N, const int* __restrict__ ptr, const int* __restrict__ col,
                                                      const double* __restrict__ val, double* __restrict__ D) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    double* row = D + (long long)r * N;
    for (int c = 0; c < N; ++c) row[c] = 0.0;
    for (int q = ptr[r]; q < ptr[r + 1]; ++q) row[col[q]] = val[q];
}

}  // namespace

void launch_csr_mv(int rows, const int* ptr, const int* col, const double* val, const double* x, const double* z,
                   double* y, double a, double c, hipStream_t st) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_csr_mv, dim3(blocks((long long)rows * LPR)), dim3(TPB), 0, st, rows, ptr, col, val, x, z, y,
                       a, c);
}

void launch_csr_assemble(int nnz, const double* val0, const int* kptr, const int* ktri, const double* kcoef,
                         const double* kinv, double* val, hipStream_t st) {
    if (nnz <= 0) return;
    hipLaunchKernelGGL(k_csr_assemble, dim3(blocks(nnz)), dim3(TPB), 0, st, nnz, val0, kptr, ktri, kcoef, kinv, val);
}

void launch_kinv_flat(long long ntri, const double* K, double Ks, int mode, double* kinv, hipStream_t st) {
    if (ntri <= 0) return;
    hipLaunchKernelGGL(k_kinv_flat, dim3(blocks(ntri)), dim3(TPB), 0, st, ntri, K, Ks, mode, kinv);
}

void launch_kinv_coarsen_flat(int nc, const double* kf, double* kc, hipStream_t st) {
    hipLaunchKernelGGL(k_kinv_coarsen_flat, dim3(blocks(2LL * nc * nc)), dim3(TPB), 0, st, nc, kf, kc);
}

void launch_patch_inverse(int np, const int* slots, const int* ptr, const int* col, const double* val, double shift,
                          double* inv, int* status, hipStream_t st) {
    if (np <= 0) return;
    hipLaunchKernelGGL(k_patch_inverse, dim3(np), dim3(64), 0, st, np, slots, ptr, col, val, shift, inv, status);
}

void launch_patch_apply(int np, const int* slots, const double* inv, const double* r, double* y, hipStream_t st) {
    if (np <= 0) return;
    hipLaunchKernelGGL(k_patch_apply, dim3(blocks((long long)np * PATCH)), dim3(TPB), 0, st, np, slots, inv, r, y);
}

void launch_patch_gather(int N, const int* dptr, const int* dlist, const double* y, const double* wgt, double omega,
                         const double* x, double* xout, hipStream_t st) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_patch_gather, dim3(blocks(N)), dim3(TPB), 0, st, N, dptr, dlist, y, wgt, omega, x, xout);
}

void launch_patch_apply_add(int npc, const int* plist, const int* slots, const double* inv, const double* r,
                            double omega, double* x, hipStream_t st) {
    if (npc <= 0) return;
    hipLaunchKernelGGL(k_patch_apply_add, dim3(blocks((long long)npc * PATCH)), dim3(TPB), 0, st, npc, plist, slots,
                       inv, r, omega, x);
}

void launch_colour_step(int npc, const int* plist, const int* crow, const int* cbeg, const int* cend,
                        const double* inv, const int* col, const double* val, const double* b, double* x,
                        double omega, bool xzero, hipStream_t st, const int* zlist, int nz) {
    if (!xzero) nz = 0;
    const unsigned npb = (unsigned)((npc + PPB_C - 1) / PPB_C), nzb = (unsigned)((nz + TPB - 1) / TPB);
    if (npb + nzb == 0) return;
    hipLaunchKernelGGL(k_colour_step, dim3(npb + nzb), dim3(TPB), 0, st, npc, plist, crow, cbeg, cend, inv, col, val,
                       b, x, omega, xzero ? 1 : 0, zlist, nz);
}

void launch_kinv_unpad(const Layout& L, const double* kinv_padded, double* flat, hipStream_t st) {
    hipLaunchKernelGGL(k_kinv_unpad, dim3(blocks(2LL * L.n * L.n)), dim3(TPB), 0, st, L, kinv_padded, flat);
}

void launch_csr_to_dense(int N, const int* ptr, const int* col, const double* val, double* D, hipStream_t st) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_csr_to_dense, dim3(blocks(N, 64)), dim3(64), 0, st, N, ptr, col, val, D);
}

}  // namespace biot
