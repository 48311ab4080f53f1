// FP64 small-matrix helpers for one 256-thread workgroup: matrix-core tile
// products with operands in LDS or global memory, Cholesky factorisation with
// inverse, Cholesky-QR orthonormalisation, block reductions.  Shared by the
// SVD kernels; each translation unit gets its own copy.
#pragma once

#include "ircur_internal.h"
#include "ircur_gptr.h"

#include <stdint.h>

namespace ircur {

namespace {

constexpr int NT = 256;
typedef double d4 __attribute__((ext_vector_type(4)));

// Factor and per-row arrays in global memory, double or float (F32 and BF16
// modes); typed global so that no generic access is generated.
__device__ __forceinline__ double fget(const void* p, int64_t i, int dt) {
    if (dt == 0) return ((const __attribute__((address_space(1))) double*)p)[i];
    return (double)((const __attribute__((address_space(1))) float*)p)[i];
}
__device__ __forceinline__ void fput(void* p, int64_t i, double v, int dt) {
    if (dt == 0) ((__attribute__((address_space(1))) double*)p)[i] = v;
    else ((__attribute__((address_space(1))) float*)p)[i] = (float)v;
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

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum_d(v);
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

// Lane permutations within rows of 16 lanes (DPP) applied to a double.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over each row of 16 lanes, the same value in every lane of the row:
// pairs, quads, half rows and rows by DPP permutations (quad_perm [1,0,3,2],
// [2,3,0,1], row_half_mirror, row_mirror).
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return v;
}

// LDS view of a pointer into the kernel's shared memory: helpers that are not
// inlined receive generic pointers, and generic (flat) accesses are slower
// than LDS ones and hold up the waits for other memory results.
typedef __attribute__((address_space(3))) double ldouble;
__device__ __forceinline__ ldouble* lp(double* p) { return (ldouble*)p; }
__device__ __forceinline__ const ldouble* lp(const double* p) { return (const ldouble*)p; }

// 1/sqrt(d) for a positive normal d: the hardware estimate refined by two
// Newton steps y <- y + y (1 - d y^2) / 2 (each doubles the correct bits; the
// result is within an ulp or two of the rounded value).  Shorter in dependent
// operations than a correctly rounded square root followed by a division.
__device__ __forceinline__ double rsqrt_d(double d) {
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = __builtin_fma(-d * y, y, 1.0);
        y = __builtin_fma(0.5 * y, e, y);
    }
    return y;
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
// Linv = L^-1, by the first wave: lane i holds row i of the trailing matrix
// (row i of L once factored) and column i of Linv.  Step j takes the pivot
// from lane j, scales column j, and publishes it in LDS (one write per lane,
// one broadcast read of the column per lane); with L[k][j] every lane applies
// the rank-1 update a[i][k] -= L[i][j] L[k][j] (k > j) and the forward
// elimination of column j of [L | I] on its column of Linv (x[j] *= 1/L[j][j],
// then x[k] -= L[k][j] x[j]).  One LDS round trip per step; the wave's LDS
// operations complete in program order and a wave barrier keeps the compiler
// from moving a lane's reads above the other lanes' writes.  The steps carry
// no lane-dependent selects: the entries above the diagonal of a finished row
// go on being updated but are never read, and the diagonal (the pivot) is
// kept in LDS and put in place when L is stored.  The whole wave runs every
// step (lanes >= P shadow row P - 1 and store nothing).  A pivot <= tol *
// max_j G_jj marks a dependent direction: its column of L and row of Linv are
// zero and dead[j] = 1.  G, L, Linv are P x P in LDS; L serves as the
// exchange buffer and the diagonal of Linv holds the pivots until the end, so
// G may alias neither.
template <int P>
__device__ __forceinline__ void chol_inv(const double* G_, double* L_, double* Linv_, int* dead, double tol,
                                         int live = P, double* LinvT_ = nullptr) {
    static_assert(P >= 2 && P <= 64 && P % 2 == 0, "one wave holds the P rows");
    const ldouble* G = lp(G_);
    ldouble* L = lp(L_);
    ldouble* Linv = lp(Linv_);
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        const int i = l < P ? l : P - 1;    // row of the trailing matrix and of L, column of Linv
        double a[P], x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            a[k] = G[i * P + k];
            x[k] = (k == i) ? 1.0 : 0.0;
        }
        double dmax = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) dmax = fmax(dmax, readlane_d(a[j], j));
        const double thr = tol * dmax;
        ldouble* col = L;                   // row j of the buffer: column j of L
#pragma unroll
        for (int j = 0; j < P; ++j) {
            if (j >= live) {                // a column known to be zero: dead without a step
                if (l == 0) {
                    dead[j] = 1;
                    Linv[j * P + j] = 0.0;
                }
                continue;
            }
            const double d = readlane_d(a[j], j);
            const bool dj = !(d > thr);
            const double inv = dj ? 0.0 : rsqrt_d(d);
            const double piv = dj ? 0.0 : d * inv;
            a[j] *= inv;                    // L[i][j] for i > j
            x[j] *= inv;
            col[j * P + i] = a[j];          // the shadow lanes write row P - 1's value
            if (l == 0) {
                dead[j] = dj ? 1 : 0;
                Linv[j * P + j] = piv;
            }
            __builtin_amdgcn_wave_barrier();
            double lk[P];
#pragma unroll
            for (int k = j + 1; k < P; ++k) lk[k] = col[j * P + k];
#pragma unroll
            for (int k = j + 1; k < P; ++k) {
                a[k] = __builtin_fma(-a[j], lk[k], a[k]);
                x[k] = __builtin_fma(-lk[k], x[j], x[k]);
            }
        }
        __builtin_amdgcn_wave_barrier();    // the buffers are overwritten below
        const double pii = Linv[i * P + i];
        __builtin_amdgcn_wave_barrier();
        if (l < P) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                L[i * P + k] = (k < i && k < live) ? a[k] : ((k == i) ? pii : 0.0);
                Linv[k * P + i] = (i <= k && k < live) ? x[k] : 0.0;
                if (LinvT_) lp(LinvT_)[i * P + k] = (i <= k && k < live) ? x[k] : 0.0;
            }
        }
    }
    __syncthreads();
}

// Returns the number of Cholesky passes applied (1: a single pass, no column
// refilled, so Ls holds the Cholesky factor of the input's Gram matrix).
// Orthonormalise the first `live` columns of X (m16 x P, LDS, row stride P)
// in place by Cholesky QR (X <- X Linv^T with X^T X = L L^T), repeated while
// max |X^T X - I| exceeds 1e-13 (at most `passes` passes, 4 once a column
// had to be refilled).  A dependent column
// is refilled with pseudo-random entries and the pass repeated; columns at or
// past `live` stay zero.
template <int P>
__device__ __forceinline__ int orthonormalise(double* X, int m16, int rows_valid, int live, double* Gs, double* Ls,
                              double* Li, int* dead, double* scratch, double* red, uint64_t salt,
                              int passes = 4) {
    int maxp = passes;
    int done = 0;
    for (int pass = 0; pass < maxp; ++pass) {
        mm_small<P, true, false>(X, P, X, P, Gs, m16, scratch);
        if (pass > 0) {
            // orthonormality defect after a pass: stop once it is at rounding level
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
            if (!(dmax > 1e-13)) break;
        }
        chol_inv<P>(Gs, Ls, Li, dead, 1e-14, live);
        ++done;
        mm_rows<P, false, true>(X, P, Li, P, X, P, m16, P, rows_valid);
        __syncthreads();
        int nd = 0;
        for (int j = 0; j < live; ++j) nd += dead[j];
        if (nd > 0) {
            maxp = 4;   // a refilled column needs a further pass
            for (int e = threadIdx.x; e < rows_valid * P; e += NT) {
                const int c = e % P;
                if (c < live && dead[c]) X[e] = rnd_unit(salt ^ (0x5bd1e995ull * (uint64_t)(pass + 1)), (uint64_t)e);
            }
            __syncthreads();
        }
    }
    return done;
}

}  // namespace

}  // namespace ircur
