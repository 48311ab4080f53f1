// Top-r FP64 SVD of the IRCUR core M = [D - S_{k+1}]_{I,J} (sI x sJ) and the
// pseudo-inverse rule of Phase II (section 3.1: U = H_r(M), U^+ = V_r
// Sigma_r^+ W_r^T), computed on the device.
//
// Method: block subspace iteration on M^T M with a Rayleigh-Ritz step every
// iteration.  G workgroups own row blocks of M; one grid barrier per
// iteration exchanges Z = M^T M Q.  Every workgroup then holds identical
// copies of the small matrices and takes identical control-flow decisions.
//
//   Y_blk = M_blk Q                      (Q: sJ x p, orthonormal)
//   Z     = sum_blk M_blk^T Y_blk        (= M^T M Q)       -- grid barrier
//   Y^T Y = Q^T M^T M Q = E diag(lambda) E^T   (Jacobi, p x p)
//   Ritz:  sigma_i = sqrt(lambda_i), v_i = Q e_i, w_i = Y e_i / sigma_i
//   converged when ||M^T w_i - sigma_i v_i|| = ||(Z - lambda_i Q) e_i|| / sigma_i
//             <= tol * sigma_1 for every i < r
//   otherwise Q <- orth(Z E) (Cholesky QR twice, column-scaled).
//
// The warm start is the previous iteration's Ritz basis (fixed index sets),
// or B_k[:, J]^T (resampled sets), completed with pseudo-random columns.
//
// The epilogue also builds the per-row data of the fused pass: for each
// sampled row a, [A_k[I_a, :] | W_r[a, :] | Delta[a, :]] with
// Delta = A_k[I, :] - W_r Gamma and Gamma = W_r^T A_k[I, :]; for each sampled
// column b, [B_k[:, J_b] | V_r[b, :] | Delta'[b, :]] with
// Delta'[b, :] = B_k[:, J_b] - Gamma' V_r[b, :]^T and Gamma' = B_k[:, J] V_r.
#include "ircur_internal.h"

#include <stdint.h>

namespace ircur {

namespace {

constexpr int NT = 256;
constexpr int PMAX = 32;

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
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Deterministic block reductions (4 waves).
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return r;
}
__device__ double block_max(double v, double* red) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
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

// G = X^T X for X (m x p, row-major in LDS).  G is written full (symmetric).
__device__ void gram(const double* X, int m, int p, double* G, double* red) {
    const int np = p * (p + 1) / 2;
    int nch = NT / np;
    if (nch < 1) nch = 1;
    if (nch > 8) nch = 8;
    const int tid = threadIdx.x;
    if (nch > 1) {
        // thread -> (pair, chunk); partial sums in red[pair * nch + chunk]
        if (tid < np * nch) {
            const int e = tid / nch, ch = tid - e * nch;
            int i = 0, rem = e;
            while (rem >= p - i) { rem -= p - i; ++i; }
            const int j = i + rem;
            double s = 0.0;
            for (int b = ch; b < m; b += nch) s = __builtin_fma(X[b * p + i], X[b * p + j], s);
            red[tid] = s;
        }
        __syncthreads();
        if (tid < np) {
            int i = 0, rem = tid;
            while (rem >= p - i) { rem -= p - i; ++i; }
            const int j = i + rem;
            double s = 0.0;
            for (int ch = 0; ch < nch; ++ch) s += red[tid * nch + ch];
            G[i * p + j] = s;
            G[j * p + i] = s;
        }
        __syncthreads();
    } else {
        for (int e = tid; e < np; e += NT) {
            int i = 0, rem = e;
            while (rem >= p - i) { rem -= p - i; ++i; }
            const int j = i + rem;
            double s = 0.0;
            for (int b = 0; b < m; ++b) s = __builtin_fma(X[b * p + i], X[b * p + j], s);
            G[i * p + j] = s;
            G[j * p + i] = s;
        }
        __syncthreads();
    }
}

// Orthonormalise the columns of X (m x p, LDS) in place: Cholesky QR applied
// twice to the column-scaled matrix.  A column that is (numerically) in the
// span of the earlier ones is refilled with pseudo-random entries after the
// first pass and set to zero if it is still dependent after the second.
__device__ void cholqr2(double* X, int m, int p, double* G, double* L, double* dinv,
                        int* dead, double* red, uint64_t salt) {
    const int tid = threadIdx.x;
    for (int pass = 0; pass < 2; ++pass) {
        gram(X, m, p, G, red);
        if (tid < p) {
            const double g = G[tid * p + tid];
            dinv[tid] = (g > 0.0 && __builtin_isfinite(g)) ? 1.0 / __builtin_sqrt(g) : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < p * p; e += NT) {
            const int i = e / p, j = e - i * p;
            G[e] *= dinv[i] * dinv[j];
            L[e] = 0.0;
        }
        __syncthreads();
        for (int j = 0; j < p; ++j) {
            if (tid == 0) {
                double d = G[j * p + j];
                for (int k = 0; k < j; ++k) d -= L[j * p + k] * L[j * p + k];
                const bool dj = !(dinv[j] > 0.0) || !(d > 1e-12);
                dead[j] = dj ? 1 : 0;
                L[j * p + j] = dj ? 0.0 : __builtin_sqrt(d);
            }
            __syncthreads();
            if (tid > j && tid < p) {
                const int i = tid;
                double v = 0.0;
                if (!dead[j]) {
                    v = G[i * p + j];
                    for (int k = 0; k < j; ++k) v -= L[i * p + k] * L[j * p + k];
                    v /= L[j * p + j];
                }
                L[i * p + j] = v;
            }
            __syncthreads();
        }
        // X <- X diag(dinv) L^{-T}  (row-wise forward substitution)
        for (int b = tid; b < m; b += NT) {
            double* x = X + (size_t)b * p;   // x_k is replaced by z_k once used
            for (int j = 0; j < p; ++j) {
                double y = x[j] * dinv[j];
                for (int k = 0; k < j; ++k) y -= x[k] * L[j * p + k];
                x[j] = dead[j] ? 0.0 : y / L[j * p + j];
            }
        }
        __syncthreads();
        if (pass == 0) {
            for (int e = tid; e < m * p; e += NT) {
                const int j = e % p;
                if (dead[j]) X[e] = rnd_unit(salt ^ 0x5bd1e995ull, (uint64_t)e);
            }
            __syncthreads();
        }
    }
}

// Symmetric eigendecomposition of A (p x p, LDS) by cyclic Jacobi with a
// round-robin parallel ordering.  On return lam holds the eigenvalues in
// descending order and E (p x p, row-major) the eigenvectors as columns.
__device__ void jacobi_eig(double* A, int p, double* E, double* lam, double* cs, int* pidx,
                           double* tmp, double* red) {
    const int tid = threadIdx.x;
    for (int e = tid; e < p * p; e += NT) E[e] = (e / p == e % p) ? 1.0 : 0.0;
    __syncthreads();
    const int pe = p + (p & 1);
    const int half = pe / 2;
    for (int sweep = 0; sweep < 40; ++sweep) {
        // converged when every off-diagonal entry is negligible against its
        // diagonal pair or against the largest diagonal entry
        double dmax = 0.0;
        for (int i = tid; i < p; i += NT) dmax = fmax(dmax, fabs(A[i * p + i]));
        dmax = block_max(dmax, red);
        double off = 0.0;
        for (int e = tid; e < p * p; e += NT) {
            const int i = e / p, j = e - i * p;
            if (i < j) {
                const double aij = fabs(A[e]);
                // below the rounding level of the largest entry nothing is left to do
                if (aij > 1e-15 * __builtin_sqrt(fabs(A[i * p + i] * A[j * p + j])) &&
                    aij > (double)p * 2.220446049250313e-16 * dmax)
                    off = 1.0;
            }
        }
        off = block_max(off, red);
        if (!(off > 0.0)) break;
        for (int rnd = 0; rnd < pe - 1; ++rnd) {
            if (tid < half) {
                int i, j;
                if (tid == 0) { i = rnd; j = pe - 1; }
                else { i = (rnd + tid) % (pe - 1); j = (rnd - tid + (pe - 1)) % (pe - 1); }
                if (i > j) { const int t = i; i = j; j = t; }
                double c = 1.0, s = 0.0;
                if (j < p) {
                    const double aij = A[i * p + j];
                    const double aii = A[i * p + i], ajj = A[j * p + j];
                    if (fabs(aij) > 1e-17 * __builtin_sqrt(fabs(aii * ajj)) && fabs(aij) > 1e-300 &&
                        fabs(aij) > 1e-3 * 2.220446049250313e-16 * (fabs(aii) + fabs(ajj))) {
                        const double tau = (ajj - aii) / (2.0 * aij);
                        double t;
                        if (fabs(tau) > 1e150) t = 0.5 / tau;
                        else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + __builtin_sqrt(1.0 + tau * tau));
                        c = 1.0 / __builtin_sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                cs[2 * tid] = c; cs[2 * tid + 1] = s;
                pidx[2 * tid] = i; pidx[2 * tid + 1] = (j < p) ? j : -1;
            }
            __syncthreads();
            // rows i, j of A  <-  J^T A
            for (int e = tid; e < half * p; e += NT) {
                const int t = e / p, k = e - t * p;
                const int i = pidx[2 * t], j = pidx[2 * t + 1];
                if (j >= 0) {
                    const double c = cs[2 * t], s = cs[2 * t + 1];
                    const double x = A[i * p + k], y = A[j * p + k];
                    A[i * p + k] = c * x - s * y;
                    A[j * p + k] = s * x + c * y;
                }
            }
            __syncthreads();
            // columns i, j of A and of E  <-  (.) J
            for (int e = tid; e < 2 * half * p; e += NT) {
                const int which = e / (half * p);
                const int e2 = e - which * half * p;
                const int t = e2 / p, k = e2 - t * p;
                const int i = pidx[2 * t], j = pidx[2 * t + 1];
                if (j >= 0) {
                    double* Mx = which ? E : A;
                    const double c = cs[2 * t], s = cs[2 * t + 1];
                    const double x = Mx[k * p + i], y = Mx[k * p + j];
                    Mx[k * p + i] = c * x - s * y;
                    Mx[k * p + j] = s * x + c * y;
                }
            }
            __syncthreads();
        }
    }
    // sort descending: rank of each eigenvalue
    if (tid < p) {
        const double li = A[tid * p + tid];
        int rank = 0;
        for (int j = 0; j < p; ++j) {
            const double lj = A[j * p + j];
            if (lj > li || (lj == li && j < tid)) ++rank;
        }
        pidx[tid] = rank;
    }
    __syncthreads();
    for (int e = tid; e < p * p; e += NT) {
        const int k = e / p, i = e - k * p;      // E[k][i] -> tmp[k][rank(i)]
        tmp[k * p + pidx[i]] = E[e];
    }
    if (tid < p) lam[pidx[tid]] = A[tid * p + tid];
    __syncthreads();
    for (int e = tid; e < p * p; e += NT) E[e] = tmp[e];
    __syncthreads();
}

}  // namespace

size_t svd_lds_bytes(int sJ, int p, int bs, int R) {
    const int pw = p > R ? p : R;
    size_t d = 0;
    d += (size_t)bs * sJ;         // M block
    d += (size_t)sJ * pw;         // Q (later: V_r)
    d += (size_t)sJ * pw;         // Z (later: staged B_k[:, J])
    d += (size_t)bs * pw;         // Y block
    d += 4 * (size_t)p * p;       // Gr, E, L, tmp
    d += 4 * PMAX;                // lam, dinv, cs
    d += NT;                      // red
    d += 2 * (size_t)R * R;       // Gamma, Gamma'
    d += (size_t)bs * R;          // staged A_k[I_blk, :]
    d += (size_t)bs * R;          // W block
    size_t bytes = d * sizeof(double);
    bytes += (size_t)(sJ + bs + 2 * PMAX) * sizeof(int);
    return bytes;
}

namespace {

// Loads of a gather loop are issued in batches of 8 per thread before any of
// them is consumed, so a batch costs one memory latency.
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

// out[e] = sum_g src[g * stride + e] for e < total, g in a fixed order; the
// G loads of an element are independent and issued together.
template <int G>
__device__ __forceinline__ void reduce_parts(const double* __restrict__ src, size_t stride, int total,
                                             double* out) {
    for (int e = threadIdx.x; e < total; e += NT) {
        double v[G];
#pragma unroll
        for (int g = 0; g < G; ++g) v[g] = src[(size_t)g * stride + e];
        double s = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) s += v[g];
        out[e] = s;
    }
}

}  // namespace

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

template <int G>
__global__ __launch_bounds__(256) void svd_topr_kernel(SvdArgs a) {
    if (a.st->stop) return;
#ifdef IRCUR_PHASE_PROFILE
    uint64_t t_prev = __builtin_amdgcn_s_memrealtime();
#endif
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int sI = a.sI, sJ = a.sJ, p = a.p, r = a.r, R = a.R;
    const int pw = p > R ? p : R;
    const int wg = blockIdx.x;
    const int bsz = a.bs;
    const int a0 = wg * bsz;
    int nb = sI - a0;
    if (nb > bsz) nb = bsz;
    if (nb < 0) nb = 0;

    double* Mb = smem;                          // nb x sJ
    double* Q = Mb + (size_t)bsz * sJ;
    double* Z = Q + (size_t)sJ * pw;
    double* Y = Z + (size_t)sJ * pw;
    double* Gr = Y + (size_t)bsz * pw;
    double* E = Gr + p * p;
    double* L = E + p * p;
    double* tmp = L + p * p;
    double* lam = tmp + p * p;
    double* dinv = lam + PMAX;
    double* cs = dinv + PMAX;
    double* red = cs + 2 * PMAX;
    double* gam = red + NT;                     // R x R
    double* gam2 = gam + R * R;                 // R x R
    double* Ast = gam2 + R * R;                 // bs x R
    double* Wb = Ast + (size_t)bsz * R;         // bs x R
    int* Jl = (int*)(Wb + (size_t)bsz * R);     // sJ
    int* Il = Jl + sJ;                          // bs
    int* dead = Il + bsz;                       // PMAX
    int* pidx = dead + PMAX;                    // PMAX

    uint32_t nbar = 0;
    const int64_t n1 = a.n1, n2 = a.n2;
    const int fd = (a.warm >> 8) & 1;   // 0: double factors, 1: float factors
    const int warm = a.warm & 0xff;
    const double* __restrict__ Mg = a.M;

    // ---- stage indices and the M block; warm start --------------------------
    for (int b = tid; b < sJ; b += NT) Jl[b] = a.J[b];
    for (int ar = tid; ar < nb; ar += NT) Il[ar] = a.I[a0 + ar];
    batched(nb * sJ, [&](int e) { return Mg[(size_t)a0 * sJ + e]; }, [&](int e, double v) { Mb[e] = v; });
    __syncthreads();
    if (warm == 1) {
        batched(sJ * p, [&](int e) { return a.prevV[e]; }, [&](int e, double v) { Q[e] = v; });
    } else {
        batched(sJ * p,
                [&](int e) {
                    const int b = e / p, c = e - b * p;
                    if (warm == 2 && c < r) return fget(a.B, (int64_t)c * n2 + Jl[b], fd);
                    return rnd_unit(a.salt, (uint64_t)e);
                },
                [&](int e, double v) { Q[e] = v; });
    }
    __syncthreads();
    PHASE(0);
    cholqr2(Q, sJ, p, Gr, L, dinv, dead, red, a.salt + 17);
    PHASE(1);

    int it = 0;
    bool conv = false;
    double maxres = 0.0;
    for (;;) {
        // Y_blk = M_blk Q   (two rows per thread item, both from LDS)
        for (int e = tid; e < nb * p; e += NT) {
            const int ar = e / p, c = e - ar * p;
            const double* mrow = Mb + (size_t)ar * sJ;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int b = 0;
            for (; b + 3 < sJ; b += 4) {
                s0 = __builtin_fma(mrow[b], Q[b * p + c], s0);
                s1 = __builtin_fma(mrow[b + 1], Q[(b + 1) * p + c], s1);
                s2 = __builtin_fma(mrow[b + 2], Q[(b + 2) * p + c], s2);
                s3 = __builtin_fma(mrow[b + 3], Q[(b + 3) * p + c], s3);
            }
            for (; b < sJ; ++b) s0 = __builtin_fma(mrow[b], Q[b * p + c], s0);
            Y[ar * p + c] = (s0 + s1) + (s2 + s3);
        }
        __syncthreads();
        PHASE(2);
        // Z partial = M_blk^T Y_blk, Gram partial = Y_blk^T Y_blk
        double* Zp = a.Zp + (size_t)wg * sJ * p;
        for (int e = tid; e < sJ * p; e += NT) {
            const int b = e / p, c = e - b * p;
            double s0 = 0.0, s1 = 0.0;
            int ar = 0;
            for (; ar + 1 < nb; ar += 2) {
                s0 = __builtin_fma(Mb[(size_t)ar * sJ + b], Y[ar * p + c], s0);
                s1 = __builtin_fma(Mb[(size_t)(ar + 1) * sJ + b], Y[(ar + 1) * p + c], s1);
            }
            if (ar < nb) s0 = __builtin_fma(Mb[(size_t)ar * sJ + b], Y[ar * p + c], s0);
            Zp[e] = s0 + s1;
        }
        double* Gp = a.Gp + (size_t)wg * p * p;
        for (int e = tid; e < p * p; e += NT) {
            const int i = e / p, j = e - i * p;
            double s = 0.0;
            for (int ar = 0; ar < nb; ++ar) s = __builtin_fma(Y[ar * p + i], Y[ar * p + j], s);
            Gp[e] = s;
        }
        PHASE(3);
        ++nbar;
        grid_barrier(&a.st->bar_ctr, nbar * (uint32_t)G, &a.st->svd_fail);
        PHASE(4);
        reduce_parts<G>(a.Zp, (size_t)sJ * p, sJ * p, Z);
        reduce_parts<G>(a.Gp, (size_t)p * p, p * p, Gr);
        __syncthreads();
        // symmetrise (partials are symmetric up to the summation order)
        for (int e = tid; e < p * p; e += NT) {
            const int i = e / p, j = e - i * p;
            if (i < j) { const double v = 0.5 * (Gr[e] + Gr[j * p + i]); Gr[e] = v; Gr[j * p + i] = v; }
        }
        __syncthreads();
        PHASE(5);
        jacobi_eig(Gr, p, E, lam, cs, pidx, tmp, red);
        PHASE(6);
        ++it;
        // residual of the top r Ritz triplets
        const double lam0 = lam[0] > 0.0 ? lam[0] : 0.0;
        const double sig0 = __builtin_sqrt(lam0);
        const double negl = (double)(sI > sJ ? sI : sJ) * 2.220446049250313e-16 * sig0;
        int nbp = NT / r;
        if (nbp < 1) nbp = 1;
        double part = 0.0;
        if (tid < r * nbp) {
            const int i = tid / nbp, ch = tid - i * nbp;
            const double li = lam[i];
            for (int b = ch; b < sJ; b += nbp) {
                double t = 0.0;
                for (int c = 0; c < p; ++c) t = __builtin_fma(Z[b * p + c] - li * Q[b * p + c], E[c * p + i], t);
                part = __builtin_fma(t, t, part);
            }
        }
        red[tid] = part;
        __syncthreads();
        if (tid < r) {
            double s = 0.0;
            for (int ch = 0; ch < nbp; ++ch) s += red[tid * nbp + ch];
            const double si = __builtin_sqrt(lam[tid] > 0.0 ? lam[tid] : 0.0);
            tmp[tid] = (si > negl && sig0 > 0.0) ? __builtin_sqrt(s) / si / sig0 : 0.0;
        }
        __syncthreads();
        maxres = 0.0;
        for (int i = 0; i < r; ++i) maxres = fmax(maxres, tmp[i]);
        __syncthreads();
        conv = !(maxres > a.tol);
        PHASE(7);
        if (conv || it >= a.max_it) break;
        // Q <- orth(Z E)
        for (int e = tid; e < sJ * p; e += NT) {
            const int b = e / p, c = e - b * p;
            double s = 0.0;
            for (int k = 0; k < p; ++k) s = __builtin_fma(Z[b * p + k], E[k * p + c], s);
            Q[e] = s;
        }
        __syncthreads();
        cholqr2(Q, sJ, p, Gr, L, dinv, dead, red, a.salt + 1000003ull * (uint64_t)it);
        PHASE(8);
    }

    // ---- epilogue ---------------------------------------------------------
    // sigma, keep rule (pinv: sigma_i > max(sI, sJ) * 2^-52 * sigma_1)
    const double sig0 = __builtin_sqrt(lam[0] > 0.0 ? lam[0] : 0.0);
    const double tolk = (double)(sI > sJ ? sI : sJ) * 2.220446049250313e-16 * sig0;
    if (tid < PMAX) dinv[tid] = 0.0;      // 1/sigma for kept components
    __syncthreads();
    if (tid < r) {
        const double si = __builtin_sqrt(lam[tid] > 0.0 ? lam[tid] : 0.0);
        dinv[tid] = (sig0 > 0.0 && si > tolk) ? 1.0 / si : 0.0;
    }
    // stage A_k[I_blk, :] and B_k[:, J] (independent gathers)
    batched(nb * R, [&](int e) { const int ar = e / R, c = e - ar * R; return fget(a.At, (int64_t)c * n1 + Il[ar], fd); },
            [&](int e, double v) { Ast[e] = v; });
    // Ritz basis V = Q E: full basis to prevV_out (rows b % G == wg), kept
    // columns to Z as V_r (sJ x R)
    for (int e = tid; e < sJ * p; e += NT) {
        const int b = e / p, c = e - b * p;
        double s = 0.0;
        for (int k = 0; k < p; ++k) s = __builtin_fma(Q[b * p + k], E[k * p + c], s);
        if ((b % G) == wg && a.prevV_out) a.prevV_out[e] = s;
        Z[e] = s;
    }
    __syncthreads();
    double* Vr = Q;            // sJ x R (Q no longer needed)
    for (int e = tid; e < sJ * R; e += NT) {
        const int b = e / R, c = e - b * R;
        Vr[e] = (c < r && dinv[c] > 0.0) ? Z[b * p + c] : 0.0;
    }
    __syncthreads();
    double* Bst = Z;           // R x sJ
    batched(R * sJ, [&](int e) { const int c = e / sJ, b = e - c * sJ; return fget(a.B, (int64_t)c * n2 + Jl[b], fd); },
            [&](int e, double v) { Bst[e] = v; });
    // W block (nb x R): w_i = Y e_i / sigma_i for kept components
    for (int e = tid; e < nb * R; e += NT) {
        const int ar = e / R, c = e - ar * R;
        double s = 0.0;
        if (c < r && dinv[c] > 0.0) {
            for (int k = 0; k < p; ++k) s = __builtin_fma(Y[ar * p + k], E[k * p + c], s);
            s *= dinv[c];
        }
        Wb[e] = s;
    }
    __syncthreads();
    // Gamma partial (R x R): sum_a W[a][i] A[I_a][c]
    double* Tp = a.Tp + (size_t)wg * R * R;
    for (int e = tid; e < R * R; e += NT) {
        const int i = e / R, c = e - i * R;
        double s = 0.0;
        for (int ar = 0; ar < nb; ++ar) s = __builtin_fma(Wb[ar * R + i], Ast[ar * R + c], s);
        Tp[e] = s;
    }
    // Gamma' (R x R): Gamma'[c][i] = sum_b B[c][J_b] V[b][i]
    for (int e = tid; e < R * R; e += NT) {
        const int c = e / R, i = e - c * R;
        double s = 0.0;
        for (int b = 0; b < sJ; ++b) s = __builtin_fma(Bst[c * sJ + b], Vr[b * R + i], s);
        gam2[e] = s;
    }
    PHASE(9);
    ++nbar;
    grid_barrier(&a.st->bar_ctr, nbar * (uint32_t)G, &a.st->svd_fail);
    PHASE(10);
    reduce_parts<G>(a.Tp, (size_t)R * R, R * R, gam);
    __syncthreads();
    // rowI for this block: [A_k[I_a,:] | W[a,:] | A_k[I_a,:] - (W Gamma)[a,:]]
    for (int e = tid; e < nb * R; e += NT) {
        const int ar = e / R, c = e - ar * R;
        double s = 0.0;
        for (int i = 0; i < R; ++i) s = __builtin_fma(Wb[ar * R + i], gam[i * R + c], s);
        const int64_t base = (int64_t)(a0 + ar) * a.qs;
        fput(a.rowI, base + c, Ast[e], fd);
        fput(a.rowI, base + R + c, Wb[e], fd);
        fput(a.rowI, base + 2 * R + c, Ast[e] - s, fd);
        a.W[(int64_t)(a0 + ar) * R + c] = Wb[e];
    }
    // rowJ, rows b with b % G == wg: [B_k[:,J_b] | V[b,:] | B_k[:,J_b] - (Gamma' V^T)[:, b]]
    for (int e = tid; e < sJ * R; e += NT) {
        const int b = e / R, c = e - b * R;
        if ((b % G) != wg) continue;
        double s = 0.0;
        for (int i = 0; i < R; ++i) s = __builtin_fma(gam2[c * R + i], Vr[b * R + i], s);
        const int64_t base = (int64_t)b * a.qs;
        fput(a.rowJ, base + c, Bst[c * sJ + b], fd);
        fput(a.rowJ, base + R + c, Vr[e], fd);
        fput(a.rowJ, base + 2 * R + c, Bst[c * sJ + b] - s, fd);
        a.V[e] = Vr[e];
    }
    if (wg == 0) {
        for (int e = tid; e < R * R; e += NT) {
            const int c = e / R, d = e - c * R;
            fput(a.GmI, e, gam[e], fd);             // Gamma[c][d]
            fput(a.GmJ, e, gam2[d * R + c], fd);    // Gamma'[d][c]
        }
        if (tid < R) {
            const double si = (tid < r) ? __builtin_sqrt(lam[tid] > 0.0 ? lam[tid] : 0.0) : 0.0;
            a.sigma[tid] = (tid < r && dinv[tid] > 0.0) ? si : 0.0;
            fput(a.scaleJ, tid, (tid < r) ? dinv[tid] : 0.0, fd);
        }
        if (tid == 0) {
            int kept = 0;
            for (int i = 0; i < r; ++i) kept += dinv[i] > 0.0 ? 1 : 0;
            a.info->iters = it;
            a.info->kept = kept;
            a.info->resid = maxres;
            a.info->gap = (p > r && lam[r - 1] > 0.0) ? __builtin_sqrt((lam[r] > 0.0 ? lam[r] : 0.0) / lam[r - 1]) : 0.0;
            if (!conv) a.st->svd_capped = 1;
            if (kept < r && sig0 > 0.0) a.st->rank_drop = 1;
        }
    }
    PHASE(11);
}

hipError_t launch_svd(const SvdArgs& a, int dtype, size_t lds_bytes, hipStream_t s) {
    SvdArgs b = a;
    b.warm = (a.warm & 0xff) | ((dtype == 0 ? 0 : 1) << 8);
    const void* fn;
    switch (a.G) {
        case 8: fn = (const void*)svd_topr_kernel<8>; break;
        case 16: fn = (const void*)svd_topr_kernel<16>; break;
        case 32: fn = (const void*)svd_topr_kernel<32>; break;
        default: return hipErrorInvalidValue;
    }
    // the attribute is raised once per instantiation to the 160 KiB maximum
    static bool attr_set[3] = {false, false, false};
    const int gi = a.G == 8 ? 0 : (a.G == 16 ? 1 : 2);
    if (!attr_set[gi]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set[gi] = true;
    }
    (void)lds_bytes;
    switch (a.G) {
        case 8: svd_topr_kernel<8><<<8, NT, lds_bytes, s>>>(b); break;
        case 16: svd_topr_kernel<16><<<16, NT, lds_bytes, s>>>(b); break;
        default: svd_topr_kernel<32><<<32, NT, lds_bytes, s>>>(b); break;
    }
    return hipGetLastError();
}

hipError_t launch_set_bar(DevState* st, hipStream_t s) {
    return hipMemsetAsync(&st->bar_ctr, 0, sizeof(uint32_t), s);
}

}  // namespace ircur
