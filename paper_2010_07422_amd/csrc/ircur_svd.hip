// Phase II of Algorithm 1 on the device, in FP64: the rank-r truncation
// U = H_r(M) of the core M = [D - S_{k+1}]_{I,J} (sI x sJ) and its
// pseudo-inverse (section 3.1), prepared for the fused pass.
//
// If the columns of Q (sJ x r) span the top-r right singular subspace of M
// and Y = M Q, then U^+ = V_r Sigma_r^-1 W_r^T = Q (Y^T Y)^-1 Y^T exactly,
// whatever basis Q is.  With the Cholesky factor Y^T Y = Ly Ly^T:
//
//     Wt = Y Ly^-T          orthonormal basis of the top-r left subspace
//     B_{k+1} = Wt^T R      (R = [D - S_{k+1}]_{I,:})
//     A_{k+1} = (C Q) Ly^-T (C = [D - S_{k+1}]_{:,J})
//     H_r(M)  = Wt Ly^T Q^T, so the singular values of H_r(M) are those of Ly.
//
// Q comes from subspace iteration on M^T M, G workgroups owning row blocks
// of M and one grid barrier per iteration:
//     Y = M Q,  Z = M^T Y,  Gy = Y^T Y = Q^T Z,  H = Y^T A_k[I,:]
//     converged when ||Z - Q Gy||_F <= tol ||Gy||_F  (span Q invariant)
//     else Q <- orth(Z) (Cholesky QR, repeated when orthogonality is short).
// No eigen- or singular-value decomposition is formed.  Pivots of Ly below
// a relative threshold are dropped (the pseudo-inverse rule; the threshold
// acts on squared singular values).
//
// Every product is a dense FP64 contraction on the matrix cores
// (v_mfma_f64_16x16x4f64); the r x r Cholesky factorisation and triangular
// inverse run in one wave with the matrix in registers.  Every workgroup
// holds the reduced small matrices and takes identical control-flow
// decisions.
//
// The epilogue builds the per-row data of the pass: for each sampled row a,
// [A_k[I_a, :] | Wt[a, :] | Delta[a, :]] with Delta = A_k[I,:] - Wt Gamma,
// Gamma = Wt^T A_k[I,:] = Ly^-1 H; for each sampled column b,
// [B_k[:, J_b] | Q[b, :] | Delta'[b, :]] with Delta'[b,:] = B_k[:,J_b] - Gamma' Q[b,:]^T,
// Gamma' = B_k[:, J] Q; and the r x r maps Gamma, Gamma'^T and Ly^-T.
#include "ircur_internal.h"

#include <stdint.h>

namespace ircur {

namespace {

constexpr int NT = 256;
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double fget(const void* p, int64_t i, int dt) {
    if (dt == 0) return ((const double*)p)[i];
    return (double)((const float*)p)[i];   // float factors (F32 and BF16 modes)
}
__device__ __forceinline__ void fput(void* p, int64_t i, double v, int dt) {
    if (dt == 0) ((double*)p)[i] = v;
    else ((float*)p)[i] = (float)v;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double rnd_unit(uint64_t salt, uint64_t i) {
    const uint64_t h = mix64(salt + 0x9E3779B97F4A7C15ull * (i + 1));
    return (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Grid barrier over the G workgroups of this launch.  All workgroups are
// resident (G is far below the number of compute units).  The spin is
// bounded: on time-out a flag is raised and the kernel continues, so every
// wave always reaches the end of the kernel.
__device__ void grid_barrier(uint32_t* ctr, uint32_t target, int32_t* fail) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > (1u << 22)) { __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break; }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
    }
    __syncthreads();
}

// ------------------------------------------------------- MFMA (FP64) ---
// One 16 x 16 output tile, acc += op(A) op(B) over k in [k0, k1) (multiples
// of 4), operands in LDS.  Operand layout of v_mfma_f64_16x16x4f64: lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; output element v of lane l is
// C[l/16 + 4 v][l%16].
// op(A)(i, k) = TA ? A[k*lda + i] : A[i*lda + k];  op(B)(k, j) = TB ? B[j*ldb + k] : B[k*ldb + j].
template <bool TA, bool TB>
__device__ __forceinline__ d4 mm_tile(const double* A, int lda, int i0, const double* B, int ldb, int j0,
                                      int k0, int k1, d4 acc) {
    const int l = threadIdx.x & 63;
    const int ii = i0 + (l & 15), jj = j0 + (l & 15), kk = l >> 4;
    // operands of 8 k-steps are loaded before their products are issued
    for (int kb = k0; kb < k1; kb += 32) {
        double av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = kb + 4 * u;
            if (k < k1) {
                av[u] = TA ? A[(k + kk) * lda + ii] : A[ii * lda + k + kk];
                bv[u] = TB ? B[jj * ldb + k + kk] : B[(k + kk) * ldb + jj];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (kb + 4 * u < k1) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    return acc;
}

__device__ __forceinline__ void tile_store(double* C, int ldc, int i0, int j0, d4 acc, int rows_valid) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = i0 + (l >> 4) + 4 * v;
        C[i * ldc + j0 + (l & 15)] = (i < rows_valid) ? acc[v] : 0.0;
    }
}

// C (m16 x P) = op(A) op(B) over K (multiple of 4), one 16-row group (all P
// columns) per work item, the four waves taking groups round robin.  Rows of
// C at or past rows_valid are written as zero.  C may alias op(A)'s rows when
// TA is false (a group reads only its own rows before writing them).
template <int P, bool TA, bool TB>
__device__ void mm_rows(const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                        int m16, int K, int rows_valid) {
    const int w = threadIdx.x >> 6;
    for (int t = w; t < (m16 >> 4); t += 4) {
        const int i0 = t * 16;
        d4 acc0 = {0.0, 0.0, 0.0, 0.0};
        acc0 = mm_tile<TA, TB>(A, lda, i0, B, ldb, 0, 0, K, acc0);
        if (P == 32) {
            d4 acc1 = {0.0, 0.0, 0.0, 0.0};
            acc1 = mm_tile<TA, TB>(A, lda, i0, B, ldb, 16, 0, K, acc1);
            tile_store(C, ldc, i0, 0, acc0, rows_valid);
            tile_store(C, ldc, i0, 16, acc1, rows_valid);
        } else {
            tile_store(C, ldc, i0, 0, acc0, rows_valid);
        }
    }
}

// P x P result of a long contraction over K4 (multiple of 4): the four waves
// split K, the partial tiles are summed in LDS in a fixed order.
template <int P, bool TA, bool TB>
__device__ void mm_small(const double* A, int lda, const double* B, int ldb, double* C, int K4,
                         double* scratch /* 4 * P * P */) {
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int ksteps = K4 >> 2;
    const int per = (ksteps + 3) >> 2;
    const int k0 = min(ksteps, w * per) * 4, k1 = min(ksteps, (w + 1) * per) * 4;
    constexpr int nt = P / 16;
#pragma unroll
    for (int ti = 0; ti < nt; ++ti)
#pragma unroll
        for (int tj = 0; tj < nt; ++tj) {
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            acc = mm_tile<TA, TB>(A, lda, ti * 16, B, ldb, tj * 16, k0, k1, acc);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                scratch[w * P * P + (ti * 16 + (l >> 4) + 4 * v) * P + tj * 16 + (l & 15)] = acc[v];
        }
    __syncthreads();
    for (int e = threadIdx.x; e < P * P; e += NT)
        C[e] = ((scratch[e] + scratch[P * P + e]) + scratch[2 * P * P + e]) + scratch[3 * P * P + e];
    __syncthreads();
}

// ------------------------------------------------ small factorisations ---
// Cholesky G = L L^T of a P x P symmetric positive semidefinite matrix and
// Linv = L^-1, by the first wave with lane i holding row i in registers.  A
// pivot <= tol * max_j G_jj marks a dependent direction: its column of L and
// row of Linv are zero and dead[j] = 1.  G, L, Linv are P x P in LDS.
template <int P>
__device__ void chol_inv(const double* G, double* L, double* Linv, int* dead, double tol) {
    if (threadIdx.x < 64) {
        const int i = threadIdx.x;
        double a[P];
#pragma unroll
        for (int j = 0; j < P; ++j) a[j] = (i < P) ? G[i * P + j] : 0.0;
        double dmax = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) dmax = fmax(dmax, readlane_d(a[j], j));
        const double thr = tol * dmax;
        double inv_d[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const double d = readlane_d(a[j], j);
            const bool dj = !(d > thr);
            const double piv = dj ? 0.0 : __builtin_sqrt(d);
            const double inv = dj ? 0.0 : 1.0 / piv;
            inv_d[j] = inv;
            const double lij = (i > j) ? a[j] * inv : ((i == j) ? piv : 0.0);
            a[j] = lij;
#pragma unroll
            for (int k = j + 1; k < P; ++k) {
                const double lk = readlane_d(lij, k);
                if (i >= k) a[k] = __builtin_fma(-lij, lk, a[k]);
            }
            if (i == 0) dead[j] = dj ? 1 : 0;
        }
        // Linv by forward elimination on [L | I], rows in order
        double x[P];
#pragma unroll
        for (int j = 0; j < P; ++j) x[j] = (i == j) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (i == k) {
#pragma unroll
                for (int j = 0; j <= k; ++j) x[j] *= inv_d[k];
            }
            if (i > k) {
                const double lik = a[k];
#pragma unroll
                for (int j = 0; j <= k; ++j) x[j] = __builtin_fma(-lik, readlane_d(x[j], k), x[j]);
            } else {
#pragma unroll
                for (int j = 0; j <= k; ++j) (void)readlane_d(x[j], k);
            }
        }
        if (i < P) {
#pragma unroll
            for (int j = 0; j < P; ++j) {
                L[i * P + j] = (j <= i) ? a[j] : 0.0;
                Linv[i * P + j] = (j <= i) ? x[j] : 0.0;
            }
        }
    }
    __syncthreads();
}

// Orthonormalise the first `live` columns of X (m16 x P, LDS, row stride P)
// in place by Cholesky QR (X <- X Linv^T with X^T X = L L^T), repeated while
// max |X^T X - I| exceeds 1e-13 (at most three passes).  A dependent column
// is refilled with pseudo-random entries and the pass repeated; columns at or
// past `live` stay zero.
template <int P>
__device__ void orthonormalise(double* X, int m16, int rows_valid, int live, double* Gs, double* Ls,
                               double* Li, int* dead, double* scratch, double* red, uint64_t salt) {
    for (int pass = 0; pass < 4; ++pass) {
        mm_small<P, true, false>(X, P, X, P, Gs, m16, scratch);
        // orthonormality defect
        double dev = 0.0;
        for (int e = threadIdx.x; e < P * P; e += NT) {
            const int i = e / P, j = e - i * P;
            if (i < live && j < live) dev = fmax(dev, fabs(Gs[e] - (i == j ? 1.0 : 0.0)));
        }
        for (int off = 32; off >= 1; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dev;
        __syncthreads();
        const double dmax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        __syncthreads();
        if (!(dmax > 1e-13) && pass > 0) break;
        chol_inv<P>(Gs, Ls, Li, dead, 1e-14);
        mm_rows<P, false, true>(X, P, Li, P, X, P, m16, P, rows_valid);
        __syncthreads();
        int nd = 0;
        for (int j = 0; j < live; ++j) nd += dead[j];
        if (nd > 0) {
            for (int e = threadIdx.x; e < rows_valid * P; e += NT) {
                const int c = e % P;
                if (c < live && dead[c]) X[e] = rnd_unit(salt ^ (0x5bd1e995ull * (uint64_t)(pass + 1)), (uint64_t)e);
            }
            __syncthreads();
        }
    }
}

// Sum of G partials (stride apart) in a fixed order, loads issued together.
template <int G>
__device__ __forceinline__ void reduce_parts(const double* __restrict__ src, size_t stride, int total,
                                             double* out) {
    constexpr int E = G <= 8 ? 7 : (G <= 16 ? 3 : 1);   // elements per thread per batch (<= 63 loads)
    for (int e0 = threadIdx.x; e0 < total; e0 += NT * E) {
        double v[E][G];
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int e = e0 + q * NT;
#pragma unroll
            for (int g = 0; g < G; ++g) v[q][g] = (e < total) ? src[(size_t)g * stride + e] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int e = e0 + q * NT;
            double s = 0.0;
#pragma unroll
            for (int g = 0; g < G; ++g) s += v[q][g];
            if (e < total) out[e] = s;
        }
    }
}

// Gather loop with loads issued in batches of 8 per thread.
template <typename LoadF, typename StoreF>
__device__ __forceinline__ void batched(int total, LoadF load, StoreF store) {
    for (int base = threadIdx.x; base < total; base += NT * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + u * NT;
            v[u] = e < total ? load(e) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + u * NT;
            if (e < total) store(e, v[u]);
        }
    }
}

}  // namespace

// LDS layout of the kernel (doubles): Q, Z (sJ16 x P each), Y, Ab, Wb
// (bs16 x P each), 8 P x P matrices, the MFMA scratch (4 P x P), a reduction
// buffer; ints: J, I, dead.  The core block itself stays in global memory in
// the two operand-tiled layouts written by the core kernel.
size_t svd_lds_bytes(int sJ, int bs16, int P) {
    const size_t sJ16 = ((size_t)sJ + 15) / 16 * 16;
    size_t d = 0;
    d += 2 * sJ16 * P;                // Q, Z
    d += 3 * (size_t)bs16 * P;        // Y, Ab, Wb
    d += 8 * (size_t)P * P;           // Gy, H, Gs, Ls, Li, Gam, Gam2, TA
    d += 4 * (size_t)P * P;           // MFMA scratch
    d += 64;                          // reduction buffer
    d += (size_t)P * sJ16;            // B_k[:, J]
    size_t bytes = d * sizeof(double);
    bytes += (sJ16 + (size_t)bs16 + 64) * sizeof(int);
    return bytes;
}

#ifdef IRCUR_PHASE_PROFILE
#define PHASE(i)                                                              \
    do {                                                                      \
        if (blockIdx.x == 0 && threadIdx.x == 0) {                            \
            const uint64_t t_ = __builtin_amdgcn_s_memrealtime();             \
            a.st->phase[i] += t_ - t_prev;                                    \
            t_prev = t_;                                                      \
        }                                                                     \
    } while (0)
#else
#define PHASE(i) do { } while (0)
#endif

template <int G, int P>
__global__ __launch_bounds__(256) void svd_sub_kernel(SvdArgs a) {
    if (a.st->stop) return;
#ifdef IRCUR_PHASE_PROFILE
    uint64_t t_prev = __builtin_amdgcn_s_memrealtime();
#endif
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int sI = a.sI, sJ = a.sJ, r = a.r, R = a.R;
    const int wg = blockIdx.x;
    const int bs16 = a.bs;              // rows of M per workgroup, a multiple of 16
    const int sJ16 = ((sJ + 15) / 16) * 16;
    const int sI16 = ((sI + 15) / 16) * 16;
    const int KSA = sJ16 / 4;           // k-steps of the row-tiled layout
    const int KSB = sI16 / 4;           // k-steps of the column-tiled layout
    const int a0 = wg * bs16;
    int nb = sI - a0;
    if (nb > bs16) nb = bs16;
    if (nb < 0) nb = 0;
    const int nt_rows = (nb + 15) / 16;  // row tiles owned by this workgroup
    const int fd = (a.warm >> 8) & 1;   // 0: double factors, 1: float factors
    const int warm = a.warm & 0xff;
    const int64_t n1 = a.n1, n2 = a.n2;
    const int l64 = tid & 63, w4 = tid >> 6;

    double* Q = smem;
    double* Z = Q + (size_t)sJ16 * P;
    double* Y = Z + (size_t)sJ16 * P;
    double* Ab = Y + (size_t)bs16 * P;
    double* Wb = Ab + (size_t)bs16 * P;
    double* Gy = Wb + (size_t)bs16 * P;
    double* H = Gy + P * P;                     // must follow Gy (reduced together)
    double* Gs = H + P * P;
    double* Ls = Gs + P * P;
    double* Li = Ls + P * P;
    double* Gam = Li + P * P;
    double* Gam2 = Gam + P * P;
    double* TA = Gam2 + P * P;
    double* scr = TA + P * P;                   // 4 P x P
    double* red = scr + 4 * P * P;              // 64
    double* Bs = red + 64;                      // P x sJ16: B_k[c, J_b]
    const int ldm = sJ16;
    int* Jl = (int*)(Bs + (size_t)P * ldm);     // sJ16
    int* Il = Jl + sJ16;                        // bs16
    int* dead = Il + bs16;                      // 64

    uint32_t nbar = 0;

    // ---- stage ----------------------------------------------------------
    for (int b = tid; b < sJ16; b += NT) Jl[b] = b < sJ ? a.J[b] : 0;
    for (int ar = tid; ar < bs16; ar += NT) Il[ar] = ar < nb ? a.I[a0 + ar] : 0;
    __syncthreads();
    batched(bs16 * P,
            [&](int e) { const int ar = e / P, c = e - ar * P;
                         return (ar < nb && c < R) ? fget(a.At, (int64_t)c * n1 + Il[ar], fd) : 0.0; },
            [&](int e, double v) { Ab[e] = v; });
    batched(P * ldm,
            [&](int e) { const int c = e / ldm, b = e - c * ldm;
                         return (c < R && b < sJ) ? fget(a.B, (int64_t)c * n2 + Jl[b], fd) : 0.0; },
            [&](int e, double v) { Bs[e] = v; });
    __syncthreads();
    // warm start Q (sJ16 x P; columns >= r and rows >= sJ zero)
    for (int e = tid; e < sJ16 * P; e += NT) {
        const int b = e / P, c = e - b * P;
        double v = 0.0;
        if (b < sJ && c < r) {
            if (warm == 1) v = a.prevV[b * R + c];
            else if (warm == 2) v = Bs[c * ldm + b];
            else v = rnd_unit(a.salt, (uint64_t)e);
        }
        Q[e] = v;
    }
    __syncthreads();
    PHASE(0);
    if (warm != 1) orthonormalise<P>(Q, sJ16, sJ, r, Gs, Ls, Li, dead, scr, red, a.salt + 17);
    __syncthreads();
    PHASE(1);

    int it = 0;
    bool conv = false;
    double rho = 0.0;
    for (;;) {
        // Y_blk = M_blk Q (bs16 x P): row tile t of this block, A operands
        // streamed from the row-tiled copy of M (one 512-byte load per k-step)
        for (int t = w4; t < bs16 / 16; t += 4) {
            d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
            if (t < nt_rows) {
                const double* __restrict__ ma = a.MA + ((size_t)(a0 / 16 + t) * KSA) * 64 + l64;
                for (int k0 = 0; k0 < KSA; k0 += 16) {
                    double av[16], bv0[16], bv1[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int kr = 4 * (k0 + u) + (l64 >> 4);
                        const bool in = k0 + u < KSA;
                        av[u] = in ? ma[(size_t)(k0 + u) * 64] : 0.0;
                        bv0[u] = in ? Q[kr * P + (l64 & 15)] : 0.0;
                        if (P == 32) bv1[u] = in ? Q[kr * P + 16 + (l64 & 15)] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        if (k0 + u < KSA) {
                            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv0[u], acc0, 0, 0, 0);
                            if (P == 32) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv1[u], acc1, 0, 0, 0);
                        }
                    }
                }
            }
            tile_store(Y, P, t * 16, 0, acc0, nb);
            if (P == 32) tile_store(Y, P, t * 16, 16, acc1, nb);
        }
        __syncthreads();
        PHASE(2);
        // partials: Z_blk = M_blk^T Y_blk (sJ x P), A operands from the
        // column-tiled copy of M; Gy_blk = Y^T Y, H_blk = Y^T A_blk
        {
            // the wave's column tiles tj = w4, w4 + 4, ... (at most 8) share the
            // Y operand of each k-step; their A operands are loaded together
            constexpr int TMAX = 8;
            double* Zp = a.Zp + (size_t)wg * sJ * P;
            const int ks0 = a0 / 4, nks = nt_rows * 4;
            const int ntj = sJ16 / 16;
            const int mine = (ntj - w4 + 3) / 4;
            for (int tb = 0; tb < mine; tb += TMAX) {
                d4 acc0[TMAX], acc1[TMAX];
#pragma unroll
                for (int q = 0; q < TMAX; ++q) {
                    acc0[q] = d4{0.0, 0.0, 0.0, 0.0};
                    acc1[q] = d4{0.0, 0.0, 0.0, 0.0};
                }
                for (int k0 = 0; k0 < nks; k0 += 4) {
                    double av[4][TMAX], y0[4], y1[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool in = k0 + u < nks;
                        const int kr = 4 * (k0 + u) + (l64 >> 4);
                        y0[u] = in ? Y[kr * P + (l64 & 15)] : 0.0;
                        if (P == 32) y1[u] = in ? Y[kr * P + 16 + (l64 & 15)] : 0.0;
#pragma unroll
                        for (int q = 0; q < TMAX; ++q) {
                            const int tj = w4 + 4 * (tb + q);
                            av[u][q] = (in && tb + q < mine)
                                           ? a.MB[((size_t)tj * KSB + ks0 + k0 + u) * 64 + l64] : 0.0;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (k0 + u < nks) {
#pragma unroll
                            for (int q = 0; q < TMAX; ++q) {
                                if (tb + q < mine) {
                                    acc0[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][q], y0[u], acc0[q], 0, 0, 0);
                                    if (P == 32) acc1[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][q], y1[u], acc1[q], 0, 0, 0);
                                }
                            }
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < TMAX; ++q) {
                    if (tb + q >= mine) continue;
                    const int tj = w4 + 4 * (tb + q);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = tj * 16 + (l64 >> 4) + 4 * v;
                        if (i < sJ) {
                            Zp[(size_t)i * P + (l64 & 15)] = acc0[q][v];
                            if (P == 32) Zp[(size_t)i * P + 16 + (l64 & 15)] = acc1[q][v];
                        }
                    }
                }
            }
        }
        mm_small<P, true, false>(Y, P, Y, P, Gy, bs16, scr);
        mm_small<P, true, false>(Y, P, Ab, P, H, bs16, scr);
        {
            double* Gp = a.Gp + (size_t)wg * 2 * P * P;
            for (int e = tid; e < P * P; e += NT) {
                Gp[e] = Gy[e];
                Gp[P * P + e] = H[e];
            }
        }
        PHASE(3);
        ++nbar;
        grid_barrier(&a.st->bar_ctr, nbar * (uint32_t)G, &a.st->svd_fail);
        PHASE(4);
        reduce_parts<G>(a.Zp, (size_t)sJ * P, sJ * P, Z);
        reduce_parts<G>(a.Gp, (size_t)2 * P * P, 2 * P * P, Gy);   // Gy then H (adjacent in LDS)
        for (int e = tid; e < (sJ16 - sJ) * P; e += NT) Z[sJ * P + e] = 0.0;
        __syncthreads();
        PHASE(5);
        // convergence: ||Z - Q Gy||_F <= tol ||Gy||_F, Q Gy formed tile by tile
        double part = 0.0;
        for (int t = w4; t < sJ16 / 16; t += 4) {
#pragma unroll
            for (int j0 = 0; j0 < P; j0 += 16) {
                d4 acc = {0.0, 0.0, 0.0, 0.0};
                acc = mm_tile<false, false>(Q, P, t * 16, Gy, P, j0, 0, P, acc);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = t * 16 + (l64 >> 4) + 4 * v;
                    const double d = (i < sJ) ? Z[i * P + j0 + (l64 & 15)] - acc[v] : 0.0;
                    part = __builtin_fma(d, d, part);
                }
            }
        }
        double gn = 0.0;
        for (int e = tid; e < P * P; e += NT) gn = __builtin_fma(Gy[e], Gy[e], gn);
        const double num = block_sum(part, red);
        const double den = block_sum(gn, red);
        rho = den > 0.0 ? __builtin_sqrt(num / den) : 0.0;
        ++it;
        conv = !(rho > a.tol);
        PHASE(6);
        if (conv || it >= a.max_it) break;
        // Q <- orth(Z)
        for (int e = tid; e < sJ16 * P; e += NT) Q[e] = Z[e];
        __syncthreads();
        orthonormalise<P>(Q, sJ16, sJ, r, Gs, Ls, Li, dead, scr, red,
                          a.salt ^ (0x2545F4914F6CDD1Dull * (uint64_t)(it + 1)));
        PHASE(7);
    }

    // ---- epilogue ---------------------------------------------------------
    // Gy = Ly Ly^T; pivots below ptol * max are dropped (pinv rule on sigma^2)
    const double ptol = 4.0 * (double)(sI > sJ ? sI : sJ) * 2.220446049250313e-16;
    chol_inv<P>(Gy, Ls, Li, dead, ptol);
    mm_rows<P, false, true>(Y, P, Li, P, Wb, P, bs16, P, nb);     // Wt = Y Ly^-T (this block)
    // Gamma = Ly^-1 H;  TA = Ly^-T;  Kc = Ly^T  (r x r, one entry per thread)
    for (int e = tid; e < P * P; e += NT) {
        const int i = e / P, j = e - i * P;
        double g = 0.0;
        for (int k = 0; k < P; ++k) g = __builtin_fma(Li[i * P + k], H[k * P + j], g);
        Gam[e] = g;
        TA[e] = Li[j * P + i];
    }
    __syncthreads();
    // Gamma' = B_k[:, J] Q  (P x P over sJ)
    mm_small<P, false, false>(Bs, ldm, Q, P, Gam2, sJ16, scr);
    PHASE(8);
    // Delta_blk = A_blk - Wt_blk Gamma  (into Y, no longer needed)
    mm_rows<P, false, false>(Wb, P, Gam, P, Y, P, bs16, P, nb);
    __syncthreads();
    // rowI: [A_k[I_a,:] | Wt[a,:] | Delta[a,:]]
    for (int e = tid; e < nb * R; e += NT) {
        const int ar = e / R, c = e - ar * R;
        const int64_t base = (int64_t)(a0 + ar) * a.qs;
        fput(a.rowI, base + c, Ab[ar * P + c], fd);
        fput(a.rowI, base + R + c, Wb[ar * P + c], fd);
        fput(a.rowI, base + 2 * R + c, Ab[ar * P + c] - Y[ar * P + c], fd);
        a.W[(int64_t)(a0 + ar) * R + c] = Wb[ar * P + c];
    }
    // rowJ for rows b % G == wg: [B_k[:,J_b] | Q[b,:] | Delta'[b,:]]
    const int nbj = (sJ - wg + G - 1) / G;      // rows b = wg, wg + G, ...
    for (int e = tid; e < nbj * R; e += NT) {
        const int b = wg + G * (e / R), c = e % R;
        double s = 0.0;
        for (int i = 0; i < P; ++i) s = __builtin_fma(Gam2[c * P + i], Q[b * P + i], s);
        const int64_t base = (int64_t)b * a.qs;
        const double bcj = Bs[c * ldm + b];
        fput(a.rowJ, base + c, bcj, fd);
        fput(a.rowJ, base + R + c, Q[b * P + c], fd);
        fput(a.rowJ, base + 2 * R + c, bcj - s, fd);
        a.V[(int64_t)b * R + c] = Q[b * P + c];
        if (a.prevV_out) a.prevV_out[(int64_t)b * R + c] = Q[b * P + c];
    }
    if (wg == 0) {
        for (int e = tid; e < R * R; e += NT) {
            const int c = e / R, d = e - c * R;
            fput(a.GmI, e, Gam[c * P + d], fd);           // Gamma[c][d]
            fput(a.GmJ, e, Gam2[d * P + c], fd);          // Gamma'[d][c]
            fput(a.scaleJ, e, TA[c * P + d], fd);         // Ly^-T
            a.TAd[e] = TA[c * P + d];
            a.sigma[e] = Ls[d * P + c];                   // Kc = Ly^T: H_r(M) = Wt Kc Q^T
        }
        if (tid == 0) {
            int kept = 0;
            for (int i = 0; i < r; ++i) kept += dead[i] == 0 ? 1 : 0;
            a.info->iters = it;
            a.info->kept = kept;
            a.info->resid = rho;
            a.info->gap = -1.0;
            if (!conv) a.st->svd_capped = 1;
            if (kept < r && Gy[0] > 0.0) a.st->rank_drop = 1;
        }
    }
    PHASE(11);
}

hipError_t launch_svd(const SvdArgs& a, int dtype, size_t lds_bytes, hipStream_t s) {
    SvdArgs b = a;
    b.warm = (a.warm & 0xff) | ((dtype == 0 ? 0 : 1) << 8);
    const void* fn = nullptr;
    int slot = -1;
#define IRCUR_SVD_CASE(GG, PP, SL) \
    if (a.G == GG && a.p == PP) { fn = (const void*)svd_sub_kernel<GG, PP>; slot = SL; }
    IRCUR_SVD_CASE(8, 16, 0) IRCUR_SVD_CASE(16, 16, 1) IRCUR_SVD_CASE(32, 16, 2)
    IRCUR_SVD_CASE(8, 32, 3) IRCUR_SVD_CASE(16, 32, 4) IRCUR_SVD_CASE(32, 32, 5)
#undef IRCUR_SVD_CASE
    if (!fn) return hipErrorInvalidValue;
    static bool attr_set[6] = {false, false, false, false, false, false};
    if (!attr_set[slot]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set[slot] = true;
    }
    void* args[] = {&b};
    return hipLaunchKernel(fn, dim3(a.G), dim3(NT), args, lds_bytes, s);
}

hipError_t launch_set_bar(DevState* st, hipStream_t s) {
    return hipMemsetAsync(&st->bar_ctr, 0, sizeof(uint32_t), s);
}

}  // namespace ircur
