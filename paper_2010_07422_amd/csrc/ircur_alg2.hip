// Algorithm 2 (CUR to SVD, section 3.3) on the device, in FP64, for the
// factored estimate L = A I_r B (A = A_k, n1 x r; B = B_k, r x n2):
//
//   QR of A and of B^T:  Cholesky QR applied twice (the second pass corrects
//                        the rounding of the first), A = Q_A Rf_A, B^T = Q_B Rf_B;
//   SVD of Rf_A Rf_B^T:  one-sided Jacobi (Hestenes rotations) on r x r,
//                        Rf_A Rf_B^T = U_M Sigma V_M^T;
//   W = Q_A U_M,  V = Q_B V_M  (so L = W Sigma V^T).
//
// Launch sequence: gram(A, B) -> small(stage 1) -> gram(A T1, B T1') ->
// small(stage 2) -> apply.  The gram kernel sums outer products of 128-row
// chunks into per-workgroup partials; the small kernel reduces them in a
// fixed order, so results do not depend on scheduling.
#include "ircur_internal.h"

#include <stdint.h>

namespace ircur {

namespace {

constexpr int kChunkRows = 128;

__device__ __forceinline__ double fget2(const void* p, int64_t i, int dt) {
    return dt == 0 ? ((const double*)p)[i] : (double)((const float*)p)[i];
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Partial Grams: workgroup (side, w) sums y_i y_i^T over its chunks, where
// y_i = x_i T (x_i = column i of X, R entries; T = identity if null).
__global__ __launch_bounds__(256) void gram_kernel(Alg2Args a, int stage) {
    __shared__ double ys[kChunkRows][33];
    const int R = a.R;
    const int side = blockIdx.x / a.nwg, w = blockIdx.x - side * a.nwg;
    const void* X = a.X[side];
    const int64_t n = a.n[side];
    const double* T = stage == 1 ? nullptr : a.T1 + side * R * R;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t ch = w; ch * kChunkRows < n; ch += a.nwg) {
        const int t = threadIdx.x;
        if (t < kChunkRows) {
            const int64_t i = ch * kChunkRows + t;
            double x[32];
#pragma unroll
            for (int c = 0; c < 32; ++c) x[c] = (c < R && i < n) ? fget2(X, (int64_t)c * n + i, a.fdt) : 0.0;
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                if (c < R) {
                    double y = x[c];
                    if (T) {
                        y = 0.0;
#pragma unroll
                        for (int b = 0; b < 32; ++b)
                            if (b < R) y = __builtin_fma(x[b], T[b * R + c], y);
                    }
                    ys[t][c] = y;
                }
            }
        }
        __syncthreads();
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q;
            if (e < R * R) {
                const int c = e / R, d = e - c * R;
                double s = acc[q];
                for (int row = 0; row < kChunkRows; ++row) s = __builtin_fma(ys[row][c], ys[row][d], s);
                acc[q] = s;
            }
        }
        __syncthreads();
    }
    double* out = a.parts + ((size_t)side * a.nwg + w) * R * R;
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e < R * R) out[e] = acc[q];
    }
}

// Cholesky G = L L^T (R x R, LDS), thread i computing row i of each column
// in turn; a pivot <= tol * max diag marks a dependent direction (its column
// of L is zero).  Then Li = L^-1 (dead rows zero), thread m solving column m.
__device__ void chol_and_inverse(const double* G, double* L, double* Li, int R, double tol) {
    const int i = threadIdx.x;
    double dmax = 0.0;
    for (int j = 0; j < R; ++j) dmax = fmax(dmax, G[j * R + j]);
    const double thr = tol * dmax;
    for (int j = 0; j < R; ++j) {
        double d = G[j * R + j];
        for (int k = 0; k < j; ++k) d = __builtin_fma(-L[j * R + k], L[j * R + k], d);
        const bool dead = !(d > thr) || !(dmax > 0.0);
        const double piv = dead ? 0.0 : __builtin_sqrt(d);
        if (i < R) {
            double v = 0.0;
            if (i == j) v = piv;
            else if (i > j && !dead) {
                double s = G[i * R + j];
                for (int k = 0; k < j; ++k) s = __builtin_fma(-L[i * R + k], L[j * R + k], s);
                v = s / piv;
            }
            L[i * R + j] = v;
        }
        __syncthreads();
    }
    // Li column m: forward substitution on L x = e_m (dead rows give 0)
    const int m = i;
    if (m < R) {
        for (int rr = 0; rr < R; ++rr) {
            const double lrr = L[rr * R + rr];
            double s = (rr == m) ? 1.0 : 0.0;
            for (int k = 0; k < rr; ++k) s = __builtin_fma(-L[rr * R + k], Li[k * R + m], s);
            Li[rr * R + m] = lrr > 0.0 ? s / lrr : 0.0;
        }
    }
    __syncthreads();
}

// One-sided Jacobi SVD of K (R x R in LDS, only the leading r x r live) by
// the first wave, lane i owning row i of K and of Vm.  On return K holds
// U_M Sigma (columns), Vm the right vectors.
__device__ void jacobi_svd(double* K, double* Vm, int R, int r) {
    const int i = threadIdx.x;
    if (i < 64) {
        if (i < R)
            for (int c = 0; c < R; ++c) Vm[i * R + c] = (i == c) ? 1.0 : 0.0;
        for (int sweep = 0; sweep < 60; ++sweep) {
            int rotations = 0;
            for (int p = 0; p < r - 1; ++p) {
                for (int q = p + 1; q < r; ++q) {
                    const double kp = i < r ? K[i * R + p] : 0.0, kq = i < r ? K[i * R + q] : 0.0;
                    const double al = wave_sum_d(kp * kp), be = wave_sum_d(kq * kq), ga = wave_sum_d(kp * kq);
                    if (!(fabs(ga) > 1e-15 * __builtin_sqrt(al * be)) || ga == 0.0) continue;
                    ++rotations;
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + __builtin_sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / __builtin_sqrt(1.0 + t * t), sn = cs * t;
                    if (i < r) {
                        K[i * R + p] = cs * kp - sn * kq;
                        K[i * R + q] = sn * kp + cs * kq;
                        const double vp = Vm[i * R + p], vq = Vm[i * R + q];
                        Vm[i * R + p] = cs * vp - sn * vq;
                        Vm[i * R + q] = sn * vp + cs * vq;
                    }
                }
            }
            if (rotations == 0) break;
        }
    }
    __syncthreads();
}

// stage 1: reduce the Grams of A and B^T, Cholesky, T1 = L^-T per side.
// stage 2: reduce the Grams of A T1 and B^T T1', second Cholesky, the
//          triangular factors Rf = L2^T L1^T, the Jacobi SVD of Rf_A Rf_B^T,
//          the output maps Tf = T1 L2^-T U_M (side A), T1' L2'^-T V_M (side B)
//          and sigma.
__global__ __launch_bounds__(256) void small_kernel(Alg2Args a, int stage) {
    // LDS (dynamic, R x R doubles each): G[2], L[2], Li[2], K, Vm; sigma; order
    extern __shared__ __align__(16) double smem[];
    const int R = a.R, RR = R * R;
    double* G[2] = {smem, smem + RR};
    double* L[2] = {smem + 2 * RR, smem + 3 * RR};
    double* Li[2] = {smem + 4 * RR, smem + 5 * RR};
    double* K = smem + 6 * RR;
    double* Vm = smem + 7 * RR;
    double* sig = smem + 8 * RR;
    int* order = (int*)(sig + 32);
    for (int e = threadIdx.x; e < 2 * RR; e += 256) {
        const int side = e / RR, f = e - side * RR;
        const double* src = a.parts + (size_t)side * a.nwg * RR + f;
        double s = 0.0;
        for (int w = 0; w < a.nwg; ++w) s += src[(size_t)w * RR];
        G[side][f] = s;
    }
    __syncthreads();
    const double tol = 64.0 * 2.220446049250313e-16;
    for (int side = 0; side < 2; ++side) chol_and_inverse(G[side], L[side], Li[side], R, tol);
    if (stage == 1) {
        for (int e = threadIdx.x; e < 2 * RR; e += 256) {
            const int side = e / RR, f = e - side * RR, b = f / R, c = f - b * R;
            a.T1[e] = Li[side][c * R + b];   // L^-T
        }
        return;
    }
    // Rf = L2^T L1^T, with L1^T the inverse of the upper triangular
    // T1 = L1^-T (column m solves T1 y = e_m by back substitution; the Grams
    // in G are no longer needed and hold the inverses)
    if (threadIdx.x < 2 * R) {
        const int side = threadIdx.x / R, m = threadIdx.x - side * R;
        const double* T = a.T1 + side * RR;
        double* Y = G[side];
        for (int rr = R - 1; rr >= 0; --rr) {
            const double d = T[rr * R + rr];
            double s = (rr == m) ? 1.0 : 0.0;
            for (int k = rr + 1; k < R; ++k) s = __builtin_fma(-T[rr * R + k], Y[k * R + m], s);
            Y[rr * R + m] = d != 0.0 ? s / d : 0.0;
        }
    }
    __syncthreads();
    // Rf_A into Vm, Rf_B into K
    for (int e = threadIdx.x; e < 2 * RR; e += 256) {
        const int side = e / RR, f = e - side * RR, b = f / R, c = f - b * R;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s = __builtin_fma(L[side][k * R + b], G[side][k * R + c], s);
        (side == 0 ? Vm : K)[f] = s;
    }
    __syncthreads();
    // Rf_A Rf_B^T into G[0], then K
    for (int e = threadIdx.x; e < RR; e += 256) {
        const int b = e / R, c = e - b * R;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s = __builtin_fma(Vm[b * R + k], K[c * R + k], s);
        G[0][e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < RR; e += 256) K[e] = G[0][e];
    __syncthreads();
    jacobi_svd(K, Vm, R, a.r);
    // singular values and descending order
    if (threadIdx.x < 64) {
        const int c = threadIdx.x;
        double s2 = 0.0;
        for (int i = 0; i < a.r; ++i) s2 = __builtin_fma(c < R ? K[i * R + c] : 0.0, c < R ? K[i * R + c] : 0.0, s2);
        if (c < 32) sig[c] = (c < a.r) ? __builtin_sqrt(s2) : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int c = 0; c < a.r; ++c) order[c] = c;
        for (int x = 0; x < a.r; ++x)
            for (int y = x + 1; y < a.r; ++y)
                if (sig[order[y]] > sig[order[x]]) { const int t = order[x]; order[x] = order[y]; order[y] = t; }
    }
    __syncthreads();
    // U_M (column c = K[:, order[c]] / sigma), V_M likewise; into G[0], G[1]
    for (int e = threadIdx.x; e < RR; e += 256) {
        const int b = e / R, c = e - b * R;
        double u = 0.0, v = 0.0;
        if (c < a.r) {
            const int src = order[c];
            const double s = sig[src];
            const double thr = sig[order[0]] * (double)R * 2.220446049250313e-16;
            if (s > thr) {
                u = K[b * R + src] / s;
                v = Vm[b * R + src];
            }
        }
        G[0][e] = u;
        G[1][e] = v;
    }
    __syncthreads();
    // Tf_side = T1_side L2_side^-T M_side  (M_A = U_M, M_B = V_M)
    for (int e = threadIdx.x; e < 2 * RR; e += 256) {
        const int side = e / RR, f = e - side * RR, b = f / R, c = f - b * R;
        double s = 0.0;   // (L2^-T M)[b][c] = sum_k Li[k][b] M[k][c]
        for (int k = 0; k < R; ++k) s = __builtin_fma(Li[side][k * R + b], G[side][k * R + c], s);
        L[side][f] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * RR; e += 256) {
        const int side = e / RR, f = e - side * RR, b = f / R, c = f - b * R;
        const double* T = a.T1 + side * RR;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s = __builtin_fma(T[b * R + k], L[side][k * R + c], s);
        a.Tf[e] = s;
    }
    if (a.sigma_out && threadIdx.x < a.r) {
        const int c = threadIdx.x;
        const double s = sig[order[c]];
        a.sigma_out[c] = s > sig[order[0]] * (double)R * 2.220446049250313e-16 ? s : 0.0;
    }
}

// out_side[i][c] = sum_b x_i[b] Tf_side[b][c], c < r.
__global__ __launch_bounds__(256) void apply_kernel(Alg2Args a, int64_t nblk0) {
    const int side = blockIdx.x < nblk0 ? 0 : 1;
    const int64_t blk = side == 0 ? blockIdx.x : blockIdx.x - nblk0;
    const int64_t i = blk * 256 + threadIdx.x;
    const int64_t n = a.n[side];
    if (i >= n || !a.out[side]) return;
    const int R = a.R;
    const double* T = a.Tf + side * R * R;
    double x[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) x[b] = b < R ? fget2(a.X[side], (int64_t)b * n + i, a.fdt) : 0.0;
    for (int c = 0; c < a.r; ++c) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < 32; ++b)
            if (b < R) s = __builtin_fma(x[b], T[b * R + c], s);
        a.out[side][i * a.r + c] = s;
    }
}

}  // namespace

hipError_t launch_alg2(const Alg2Args& a, hipStream_t s) {
    if (a.R > 32 || a.r > a.R || a.nwg < 1) return hipErrorInvalidValue;
    const size_t lds = (size_t)8 * a.R * a.R * sizeof(double) + 32 * sizeof(double) + 32 * sizeof(int);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)small_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           96 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    gram_kernel<<<2 * a.nwg, 256, 0, s>>>(a, 1);
    small_kernel<<<1, 256, lds, s>>>(a, 1);
    gram_kernel<<<2 * a.nwg, 256, 0, s>>>(a, 2);
    small_kernel<<<1, 256, lds, s>>>(a, 2);
    const int64_t b0 = (a.n[0] + 255) / 256, b1 = (a.n[1] + 255) / 256;
    apply_kernel<<<(unsigned)(b0 + b1), 256, 0, s>>>(a, b0);
    return hipGetLastError();
}

}  // namespace ircur
