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
#include "ircur_small.h"
#include "ircur_block16.h"

#include <stdint.h>

namespace ircur {

namespace {

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

// Device-scope (all XCDs) stores and loads of the data that workgroups of
// one launch exchange across a grid barrier: written through to, and read
// from, the device-coherent level, so the barrier itself needs no cache-wide
// fence.
__device__ __forceinline__ void st_dev(gdouble* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const gdouble* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier for data exchanged with st_dev / ld_dev: every thread's stores
// have completed before the workgroup is counted, and the loads that follow
// read the device-coherent level.
__device__ void grid_barrier_dev(uint32_t* ctr, uint32_t target, int32_t* fail) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > (1u << 22)) { __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break; }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
}

// Sum of G partials (stride apart) in a fixed order, loads issued together
// (DEV: device-scope loads, for partials written with st_dev in this launch).
template <int G, bool DEV = false>
__device__ __forceinline__ void reduce_parts(const gdouble* __restrict__ src, size_t stride, int total,
                                             double* out) {
    constexpr int E = G <= 8 ? 7 : (G <= 16 ? 3 : 1);   // elements per thread per batch (<= 63 loads)
    for (int e0 = threadIdx.x; e0 < total; e0 += NT * E) {
        double v[E][G];
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int e = e0 + q * NT;
#pragma unroll
            for (int g = 0; g < G; ++g)
                v[q][g] = (e < total) ? (DEV ? ld_dev(src + (size_t)g * stride + e) : src[(size_t)g * stride + e]) : 0.0;
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
        if (wg == 0 && blockIdx.y == 0 && threadIdx.x == 0) {                 \
            const uint64_t t_ = __builtin_amdgcn_s_memrealtime();             \
            a.st->phase[i] += t_ - t_prev;                                    \
            t_prev = t_;                                                      \
        }                                                                     \
    } while (0)
#else
#define PHASE(i) do { } while (0)
#endif

template <int G, int P>
__device__ __forceinline__ void svd_body(const SvdArgs& a, const int wg) {
    if (a.st->stop) return;
#ifdef IRCUR_PHASE_PROFILE
    uint64_t t_prev = __builtin_amdgcn_s_memrealtime();
#endif
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int sI = a.sI, sJ = a.sJ, r = a.r, R = a.R;
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
        reduce_parts<G>(gp(a.Zp), (size_t)sJ * P, sJ * P, Z);
        reduce_parts<G>(gp(a.Gp), (size_t)2 * P * P, 2 * P * P, Gy);   // Gy then H (adjacent in LDS)
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
    chol_inv<P>(Gy, Ls, Li, dead, ptol, r);   // columns >= r of Y are zero
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

template <int G, int P>
__global__ __launch_bounds__(256) void svd_sub_kernel(SvdArgs a) {
    svd_body<G, P>(a, blockIdx.x);
}

// A batch of independent cores: launch (G, nb); slice y works on arr[y]
// (its own DevState and grid-barrier counter).
template <int G, int P>
__global__ __launch_bounds__(256) void svd_batch_kernel(const SvdArgs* __restrict__ arr) {
    const SvdArgs a = arr[blockIdx.y];
    svd_body<G, P>(a, blockIdx.x);
}


// ---------------------------------------------------------------------------
// Variant with the workgroup's row block of M resident in LDS (P = 16).
//
// Per subspace iteration each workgroup forms Y_blk = M_blk Q and the partial
// Z_g = M_blk^T Y_blk from LDS, then exchanges through global memory in two
// steps: after the first grid barrier it reduces only its slice of the rows
// of Z (reduce-scatter), with the small Gram matrices reduced in full; after
// the second it reads the residual parts of every slice and, if not
// converged, the whole reduced Z (all-gather) for Q <- orth(Z).  The sampled
// factor rows and columns come from compact copies written by the core
// kernel; the warm start is orthonormalised in a single Cholesky-QR pass.
size_t svdl_lds_bytes(int sJ, int bs16, int G) {
    constexpr size_t P = 16;
    const size_t sJ16 = ((size_t)sJ + 15) / 16 * 16;
    const size_t ntj = sJ16 / 16;
    const size_t tpg = (ntj + G - 1) / G;
    size_t d = 0;
    d += (size_t)bs16 * sJ16;         // M block
    d += sJ16 * P;                    // Q
    d += 3 * (size_t)bs16 * P;        // Y, Ab, Wb
    d += 8 * P * P;                   // Gy, H, Gs, Ls, Li, Gam, Gam2, TA
    d += 4 * P * P;                   // MFMA scratch
    d += 64;                          // reduction buffer
    d += tpg * 16 * P;                // this workgroup's slice of Z
    return d * sizeof(double) + 64 * sizeof(int);
}

typedef double dbl2 __attribute__((ext_vector_type(2)));

// Cholesky QR of the 16 columns of X as in orthonormalise, with the
// register factorisation chol16 (wave 0, no LDS round trip per elimination
// step) in place of chol_inv; L^-T is staged in scr (row stride XS) and the
// factor itself is not kept.  Same dead-column rule (pivot at or below 1e-14
// times the largest diagonal entry), same passes and defect test.
__device__ __forceinline__ void orthonormalise16(double* X, int m16, int rows_valid, int live, double* Gs, int* dead,
                                                 double* scr, double* red, uint64_t salt) {
    constexpr int P = 16;
    int maxp = 4;
    for (int pass = 0; pass < maxp; ++pass) {
        mm_small<P, true, false>(X, P, X, P, Gs, m16, scr);
        if (pass > 0) {
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
        chol16(Gs, P, live, 1e-14, false, nullptr, scr, dead, nullptr, scr + 512);
        mm_rows<P, false, false>(X, P, scr, XS, X, P, m16, P, rows_valid);
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

template <int G>
__device__ __forceinline__ void svdl_body(const SvdArgs& a, const int wg) {
    constexpr int P = 16;
    if (a.st->stop) return;
#ifdef IRCUR_PHASE_PROFILE
    uint64_t t_prev = __builtin_amdgcn_s_memrealtime();
#endif
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int sI = a.sI, sJ = a.sJ, r = a.r, R = a.R;
    const int bs16 = a.bs;
    const int sJ16 = ((sJ + 15) / 16) * 16;
    const int KSA = sJ16 / 4;
    const int a0 = wg * bs16;
    int nb = sI - a0;
    if (nb > bs16) nb = bs16;
    if (nb < 0) nb = 0;
    const int nt_rows = (nb + 15) / 16;
    const int ntj = sJ16 / 16;
    const int tpg = (ntj + G - 1) / G;
    const int z0 = min(wg * tpg, ntj) * 16;
    const int z1 = min(min((wg + 1) * tpg, ntj) * 16, sJ);
    const int zn = z1 > z0 ? z1 - z0 : 0;
    const int fd = (a.warm >> 8) & 1;
    const int warm = a.warm & 0xff;
    const int l64 = tid & 63, w4 = tid >> 6;

    double* Mb = smem;                          // bs16 x sJ16, row-tiled (MA) order
    double* Q = Mb + (size_t)bs16 * sJ16;
    double* Y = Q + (size_t)sJ16 * P;
    double* Ab = Y + (size_t)bs16 * P;
    double* Wb = Ab + (size_t)bs16 * P;
    double* Gy = Wb + (size_t)bs16 * P;
    double* H = Gy + P * P;                     // follows Gy (reduced together)
    double* Gs = H + P * P;
    double* Ls = Gs + P * P;
    double* Li = Ls + P * P;
    double* Gam = Li + P * P;
    double* Gam2 = Gam + P * P;
    double* TA = Gam2 + P * P;
    double* scr = TA + P * P;
    double* red = scr + 4 * P * P;
    double* Zs = red + 64;                      // tpg*16 x P
    int* dead = (int*)(Zs + (size_t)tpg * 16 * P);
    double* Zp_all = a.Zp;                      // G x sJ16 x P
    uint32_t nbar = 0;

    // ---- stage: M block, A_k[I_blk, :], warm start ------------------------
    {
        const double* __restrict__ src = a.MA + (size_t)(a0 / 16) * KSA * 64;
        const int have = nt_rows * KSA * 64;
        // 16-byte loads, up to 20 per thread in flight (one round trip for
        // blocks up to 80 KiB)
        const __attribute__((address_space(1))) dbl2* __restrict__ src2 = (const __attribute__((address_space(1))) dbl2*)src;
        dbl2* dst2 = (dbl2*)Mb;
        const int have2 = have / 2, tot2 = bs16 * sJ16 / 2;
        constexpr int V = 20;
        for (int base = tid; base < tot2; base += NT * V) {
            dbl2 v[V];
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const int e = base + u * NT;
                v[u] = e < have2 ? src2[e] : dbl2{0.0, 0.0};
            }
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const int e = base + u * NT;
                if (e < tot2) dst2[e] = v[u];
            }
        }
    }
    for (int e = tid; e < bs16 * P; e += NT) {
        const int ar = e / P;
        Ab[e] = ar < nb ? gp(a.Abc)[(size_t)(a0 + ar) * P + (e - ar * P)] : 0.0;
    }
    if (warm == 2) {
        // B_k[:, J] read along J (coalesced), written transposed
        for (int e = tid; e < sJ16 * P; e += NT) {
            const int c = e / sJ16, b = e - c * sJ16;
            Q[b * P + c] = (b < sJ && c < r) ? gp(a.Bsc)[(size_t)c * sJ16 + b] : 0.0;
        }
    } else {
        for (int e = tid; e < sJ16 * P; e += NT) {
            const int b = e / P, c = e - b * P;
            double v = 0.0;
            if (b < sJ && c < r) v = warm == 1 ? gp(a.prevV)[b * R + c] : rnd_unit(a.salt, (uint64_t)e);
            Q[e] = v;
        }
    }
    __syncthreads();
    PHASE(0);
    // with a warm start from B_k[:, J], Q0 = B_k[:, J]^T and one Cholesky-QR
    // pass Q = Q0 L0^-T, so that Gamma' = B_k[:, J] Q = Q0^T Q = L0 as long as
    // Q is not replaced: L0 is kept for the epilogue
    bool have_l0 = false;
    if (warm == 2) {
        have_l0 = orthonormalise<P>(Q, sJ16, sJ, r, Gs, Ls, Li, dead, scr, red, a.salt + 17, 1) == 1;
        for (int e = tid; e < P * P; e += NT) Gam2[e] = Ls[e];
    }
    else if (warm == 0) orthonormalise<P>(Q, sJ16, sJ, r, Gs, Ls, Li, dead, scr, red, a.salt + 17);
    __syncthreads();
    PHASE(1);

    // tolerance of this iteration: with tol_e > 0 it follows the stopping
    // residual e_k of the run (e_0 = 1), never below tol
    const double tol_k = a.tol_e > 0.0 ? fmax(a.tol, a.tol_e * (a.st->k_done > 0 ? a.st->e_last : 1.0)) : a.tol;
    int it = 0;
    bool conv = false;
    double rho = 0.0;
    for (;;) {
        // Y_blk = M_blk Q.  With fewer row tiles than waves the k range is
        // split too (ks parts per tile), so that all four waves work; the
        // parts are added in a fixed order.
        {
            const int ntl = bs16 / 16;
            const int ks = ntl >= 4 ? 1 : 4 / ntl;      // ntl * ks <= 4 partial tiles in scr
            const int kper = (KSA + ks - 1) / ks;
            for (int w = w4; w < ntl * ks; w += 4) {
                const int t = w % ntl, h = w / ntl;
                const int kb = min(KSA, h * kper), ke = min(KSA, (h + 1) * kper);
                d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
                if (t < nt_rows) {
                    const double* ma = Mb + (size_t)t * KSA * 64 + l64;
                    for (int k0 = kb; k0 < ke; k0 += 8) {
                        double av[8], bv[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const bool in = k0 + u < ke;
                            av[u] = in ? ma[(size_t)(k0 + u) * 64] : 0.0;
                            bv[u] = in ? Q[(4 * (k0 + u) + (l64 >> 4)) * P + (l64 & 15)] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < 8; u += 2) {
                            if (k0 + u < ke) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
                            if (k0 + u + 1 < ke) acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u + 1], bv[u + 1], acc2, 0, 0, 0);
                        }
                    }
                }
                acc += acc2;
                if (ks == 1) {
                    tile_store(Y, P, t * 16, 0, acc, nb);
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) scr[(size_t)w * P * P + (l64 >> 4) * P * 4 + v * P + (l64 & 15)] = acc[v];
                }
            }
            if (ks > 1) {
                __syncthreads();
                // part h of tile t sits in scr[(h * ntl + t) * P * P]: lane layout (row group, v, column)
                for (int e = tid; e < ntl * 16 * P; e += NT) {
                    const int t = e / (16 * P), rem = e - t * 16 * P;
                    const int row = rem / P, col = rem - row * P;
                    const int li = (row & 3) * P * 4 + (row >> 2) * P + col;   // v = row >> 2, group = row & 3
                    double y = 0.0;
                    for (int h = 0; h < ks; ++h) y += scr[(size_t)(h * ntl + t) * P * P + li];
                    Y[(t * 16 + row) * P + col] = (t * 16 + row < nb) ? y : 0.0;
                }
            }
        }
        __syncthreads();
        PHASE(2);
        // Z_g = M_blk^T Y_blk (sJ16 x P), column tile tj of M per work item
        {
            gdouble* Zp = gp(Zp_all) + (size_t)wg * sJ16 * P;
            const int nks = nt_rows * 4;
            for (int tj = w4; tj < ntj; tj += 4) {
                d4 acc = {0.0, 0.0, 0.0, 0.0};
                const int jj = 16 * tj + (l64 & 15);
                const double* mcol = Mb + (size_t)(jj >> 2) * 64 + ((jj & 3) << 4);
                for (int k0 = 0; k0 < nks; k0 += 8) {
                    double av[8], yv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const bool in = k0 + u < nks;
                        const int ii = 4 * (k0 + u) + (l64 >> 4);
                        av[u] = in ? mcol[(size_t)(ii >> 4) * KSA * 64 + (ii & 15)] : 0.0;
                        yv[u] = in ? Y[ii * P + (l64 & 15)] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (k0 + u < nks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], yv[u], acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) st_dev(Zp + (size_t)(16 * tj + (l64 >> 4) + 4 * v) * P + (l64 & 15), acc[v]);
            }
        }
        mm_small<P, true, false>(Y, P, Y, P, Gy, bs16, scr);
        mm_small<P, true, false>(Y, P, Ab, P, H, bs16, scr);
        {
            gdouble* Gp = gp(a.Gp) + (size_t)wg * 2 * P * P;
            for (int e = tid; e < P * P; e += NT) {
                st_dev(Gp + e, Gy[e]);
                st_dev(Gp + P * P + e, H[e]);
            }
        }
        PHASE(3);
        ++nbar;
        grid_barrier_dev(&a.st->bar_ctr, nbar * (uint32_t)G, &a.st->svd_fail);
        PHASE(4);
        // reduce-scatter: full Gy and H, this workgroup's slice of Z
        reduce_parts<G, true>(gp(a.Gp), (size_t)2 * P * P, 2 * P * P, Gy);
        reduce_parts<G, true>(gp(Zp_all) + (size_t)z0 * P, (size_t)sJ16 * P, zn * P, Zs);
        __syncthreads();
        // residual of the slice: ||Z - Q Gy||^2 over rows z0 .. z1
        double part = 0.0;
        for (int e = tid; e < zn * P; e += NT) {
            const int i = e / P, c = e - i * P;
            double q = 0.0;
#pragma unroll
            for (int d = 0; d < P; ++d) q = __builtin_fma(Q[(z0 + i) * P + d], Gy[d * P + c], q);
            const double dz = Zs[e] - q;
            part = __builtin_fma(dz, dz, part);
        }
        for (int e = tid; e < zn * P; e += NT) st_dev(gp(a.Zr) + (size_t)z0 * P + e, Zs[e]);
        const double num_s = block_sum(part, red);
        if (tid == 0) st_dev(gp(a.rp) + wg, num_s);
        PHASE(5);
        ++nbar;
        grid_barrier_dev(&a.st->bar_ctr, nbar * (uint32_t)G, &a.st->svd_fail);
        double gn = 0.0;
        for (int e = tid; e < P * P; e += NT) gn = __builtin_fma(Gy[e], Gy[e], gn);
        const double den = block_sum(gn, red);
        double num = 0.0;
        for (int g = 0; g < G; ++g) num += ld_dev(gp(a.rp) + g);
        rho = den > 0.0 ? __builtin_sqrt(num / den) : 0.0;
        ++it;
        conv = !(rho > tol_k);
        PHASE(6);
        if (conv || it >= a.max_it) break;
        // all-gather: Q <- orth(Z)
        batched(sJ16 * P, [&](int e) { return e < sJ * P ? ld_dev(gp(a.Zr) + e) : 0.0; }, [&](int e, double v) { Q[e] = v; });
        __syncthreads();
        orthonormalise16(Q, sJ16, sJ, r, Gs, dead, scr, red, a.salt ^ (0x2545F4914F6CDD1Dull * (uint64_t)(it + 1)));
        PHASE(7);
    }

    // ---- epilogue ---------------------------------------------------------
    const double ptol = 4.0 * (double)(sI > sJ ? sI : sJ) * 2.220446049250313e-16;
    chol_inv<P>(Gy, Ls, Li, dead, ptol, r);   // columns >= r of Y are zero
    mm_rows<P, false, true>(Y, P, Li, P, Wb, P, bs16, P, nb);     // Wt = Y Ly^-T (this block)
    for (int e = tid; e < P * P; e += NT) {
        const int i = e / P, j = e - i * P;
        double g = 0.0;
        for (int k = 0; k < P; ++k) g = __builtin_fma(Li[i * P + k], H[k * P + j], g);
        Gam[e] = g;
        TA[e] = Li[j * P + i];
    }
    __syncthreads();
    if (!(have_l0 && it == 1))
        mm_small<P, false, false>(a.Bsc, sJ16, Q, P, Gam2, sJ16, scr);   // Gamma' = B_k[:, J] Q
    PHASE(8);
    mm_rows<P, false, false>(Wb, P, Gam, P, Y, P, bs16, P, nb);     // Delta_blk (into Y)
    __syncthreads();
    for (int e = tid; e < nb * R; e += NT) {
        const int ar = e / R, c = e - ar * R;
        const int64_t base = (int64_t)(a0 + ar) * a.qs;
        fput(a.rowI, base + c, Ab[ar * P + c], fd);
        fput(a.rowI, base + R + c, Wb[ar * P + c], fd);
        fput(a.rowI, base + 2 * R + c, Ab[ar * P + c] - Y[ar * P + c], fd);
        gp(a.W)[(int64_t)(a0 + ar) * R + c] = Wb[ar * P + c];
    }
    const int nbj = (sJ - wg + G - 1) / G;
    for (int e = tid; e < nbj * R; e += NT) {
        const int b = wg + G * (e / R), c = e % R;
        double s = 0.0;
        for (int i = 0; i < P; ++i) s = __builtin_fma(Gam2[c * P + i], Q[b * P + i], s);
        const int64_t base = (int64_t)b * a.qs;
        const double bcj = gp(a.Bsc)[(size_t)c * sJ16 + b];
        fput(a.rowJ, base + c, bcj, fd);
        fput(a.rowJ, base + R + c, Q[b * P + c], fd);
        fput(a.rowJ, base + 2 * R + c, bcj - s, fd);
        gp(a.V)[(int64_t)b * R + c] = Q[b * P + c];
        if (a.prevV_out) gp(a.prevV_out)[(int64_t)b * R + c] = Q[b * P + c];
    }
    if (wg == 0) {
        for (int e = tid; e < R * R; e += NT) {
            const int c = e / R, d = e - c * R;
            fput(a.GmI, e, Gam[c * P + d], fd);
            fput(a.GmJ, e, Gam2[d * P + c], fd);
            fput(a.scaleJ, e, TA[c * P + d], fd);
            if (a.TAd) gp(a.TAd)[e] = TA[c * P + d];
            gp(a.sigma)[e] = Ls[d * P + c];
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

template <int G>
__global__ __launch_bounds__(256) void svdl_kernel(SvdArgs a) {
    svdl_body<G>(a, blockIdx.x);
}

template <int G>
__global__ __launch_bounds__(256) void svdl_batch_kernel(const SvdArgs* __restrict__ arr) {
    const SvdArgs a = arr[blockIdx.y];
    svdl_body<G>(a, blockIdx.x);
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

hipError_t launch_svd_batch(const SvdArgs* arr_dev, int nb, int G, int P, size_t lds_bytes, hipStream_t s) {
    const void* fn = nullptr;
    int slot = -1;
#define IRCUR_SVDB_CASE(GG, PP, SL) \
    if (G == GG && P == PP) { fn = (const void*)svd_batch_kernel<GG, PP>; slot = SL; }
    IRCUR_SVDB_CASE(1, 16, 0) IRCUR_SVDB_CASE(2, 16, 1) IRCUR_SVDB_CASE(4, 16, 2) IRCUR_SVDB_CASE(8, 16, 3)
#undef IRCUR_SVDB_CASE
    if (!fn || nb < 1) return hipErrorInvalidValue;
    static bool attr_set[4] = {false, false, false, false};
    if (!attr_set[slot]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set[slot] = true;
    }
    void* args[] = {(void*)&arr_dev};
    return hipLaunchKernel(fn, dim3(G, nb), dim3(NT), args, lds_bytes, s);
}

hipError_t launch_svdl(const SvdArgs& a, size_t lds_bytes, hipStream_t s) {
    const void* fn = nullptr;
    int slot = -1;
    if (a.G == 8) { fn = (const void*)svdl_kernel<8>; slot = 0; }
    if (a.G == 16) { fn = (const void*)svdl_kernel<16>; slot = 1; }
    if (a.G == 32) { fn = (const void*)svdl_kernel<32>; slot = 2; }
    if (!fn || a.p != 16) return hipErrorInvalidValue;
    static bool attr_set[3] = {false, false, false};
    if (!attr_set[slot]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set[slot] = true;
    }
    SvdArgs b = a;
    void* args[] = {&b};
    return hipLaunchKernel(fn, dim3(a.G), dim3(NT), args, lds_bytes, s);
}

hipError_t launch_svdl_batch(const SvdArgs* arr_dev, int nb, int G, size_t lds_bytes, hipStream_t s) {
    const void* fn = nullptr;
    int slot = -1;
    if (G == 2) { fn = (const void*)svdl_batch_kernel<2>; slot = 0; }
    if (G == 4) { fn = (const void*)svdl_batch_kernel<4>; slot = 1; }
    if (G == 8) { fn = (const void*)svdl_batch_kernel<8>; slot = 2; }
    if (!fn || nb < 1) return hipErrorInvalidValue;
    static bool attr_set[3] = {false, false, false};
    if (!attr_set[slot]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set[slot] = true;
    }
    void* args[] = {(void*)&arr_dev};
    return hipLaunchKernel(fn, dim3(G, nb), dim3(NT), args, lds_bytes, s);
}

hipError_t launch_set_bar(DevState* st, hipStream_t s) {
    return hipMemsetAsync(&st->bar_ctr, 0, sizeof(uint32_t), s);
}

}  // namespace ircur
