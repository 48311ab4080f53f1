// Small steps of the one-launch SVD on a block of 16 columns, written for
// latency (the block is small; every step sits on the critical path of an
// iteration): operands of a step are all requested before the first matrix
// core instruction that uses them, and the 16 x 16 Cholesky factorisation
// runs in the registers of one wave.
#pragma once

#include "ircur_small.h"

#include <stdint.h>

namespace ircur {

namespace {

// Row stride (doubles) of the |J| x 16 block X and of the 16 x 16 matrices
// these helpers write: 17 puts the rows of a 16 x 16 tile on distinct banks
// for reads by rows and by columns.
constexpr int XS = 17;

// Largest |J| handled (k-steps of 4 rows: 128; row tiles of 16: 32).
constexpr int KMAX = 128;
constexpr int TMAX = 32;

// Sum over the 64 lanes of a wave, the same value in every lane: the four
// row sums (row16_sum) added in row order.
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v = row16_sum(v);
    return ((readlane_d(v, 0) + readlane_d(v, 16)) + readlane_d(v, 32)) + readlane_d(v, 48);
}

// Sum over the workgroup (four waves, in wave order); red: 4 doubles.
__device__ __forceinline__ double block_sum_dpp(double v, double* red) {
    v = wave_sum_dpp(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return r;
}

// Index of the thread's wave, known to the compiler to be the same in every
// lane (branches on it are scalar).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Cholesky factorisation G = L L^T of a symmetric 16 x 16 matrix in LDS (row
// stride gs), with the inverse factor, by wave 0, as G = U D U^T (U unit lower
// triangular) followed by L = U D^1/2: the elimination needs a reciprocal of
// each pivot, the square roots are taken once at the end.  Lanes 0-15 hold the
// rows of the trailing matrix; lanes 16-31 hold the columns of U^-1 being
// solved for (forward substitution on the unit vectors).  Step j subtracts
// from every lane's row f times the pivot row (read from lane j), with
// f = v_j / d_j for both halves, so the inverse costs no extra instructions.
//
// Column j is dead when j >= live or its pivot d_j is not above thr_j:
// thr_j = tol G_jj (colrel: relative to the column's own norm, which is the
// absolute test on the column-equilibrated matrix, the factorisation being
// invariant under diagonal scaling) or thr_j = tol max_i G_ii.  A dead column
// has zero columns in L and zero rows in L^-1.
//
// Outputs in LDS (each may be null): L (row stride XS, zero above the
// diagonal and in rows >= live), T = L^-T (row stride XS), dead[0..15],
// st[0] = number of dead columns below live, st[1] and st[2] = largest and
// smallest d_j / G_jj of the kept columns among the first nst.  scr: 32
// doubles.  Called by every thread; ends with a workgroup barrier (sync), or
// without one, the other waves returning at once (the caller then places the
// barrier after their own work).
__device__ __forceinline__ void chol16(const double* G_, int gs, int live, double tol, bool colrel, double* L_,
                                       double* T_, int* dead, double* st_, double* scr_, int nst = 16,
                                       bool sync = true) {
    if (wave_id() == 0) {
        const ldouble* G = lp(G_);
        ldouble* scr = lp(scr_);
        const int l = threadIdx.x, i = l & 15;
        const bool xl = (l >> 4) == 1;
        double v[16], dg[16], fk[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const double g = G[i * gs + k];
            v[k] = xl ? (k == i ? 1.0 : 0.0) : g;
            dg[k] = G[k * gs + k];
            fk[k] = 0.0;
        }
        double dmax = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) dmax = k < live ? fmax(dmax, dg[k]) : dmax;
        uint32_t dm = 0;
        double mypiv = 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            // (no branch on live: a branch here makes every step merge the
            // whole register row; a dead step is a step with f = 0)
            const double d = readlane_d(v[j], j);
            const bool dj = j >= live || !(d > tol * (colrel ? dg[j] : dmax));
            double y = __builtin_amdgcn_rcp(d);
            y = __builtin_fma(y, __builtin_fma(-d, y, 1.0), y);
            y = __builtin_fma(y, __builtin_fma(-d, y, 1.0), y);
            const double f = v[j] * (dj ? 0.0 : y);
            fk[j] = f;
            mypiv = i == j ? (dj ? 0.0 : d) : mypiv;
            dm |= dj ? 1u << j : 0u;
#pragma unroll
            for (int k = j + 1; k < 16; ++k) v[k] = __builtin_fma(-f, readlane_d(v[k], j), v[k]);
        }
        // square roots of the pivots: lane j of the row half computes its own
        const double s = mypiv > 0.0 ? rsqrt_d(mypiv) : 0.0;
        if (l < 16) {
            scr[l] = s;
            scr[16 + l] = mypiv * s;
        }
        __builtin_amdgcn_wave_barrier();
        double sk[16], rk[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            sk[k] = scr[k];
            rk[k] = scr[16 + k];
        }
        if (l < 16) {
            if (L_) {
                ldouble* L = lp(L_);
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    L[i * XS + k] = i >= live ? 0.0 : (k < i ? fk[k] * rk[k] : (k == i ? rk[k] : 0.0));
            }
        } else if (l < 32) {
            if (T_) {
                ldouble* T = lp(T_);
#pragma unroll
                for (int k = 0; k < 16; ++k) T[i * XS + k] = v[k] * sk[k];
            }
        }
        if (dead && l >= 32 && l < 48) dead[i] = (dm >> i) & 1;
        if (st_) {
            // pivot statistics over the kept columns (lanes 0-15: their own)
            const bool kept = l < 16 && l < nst && !((dm >> i) & 1);
            const double e = kept ? mypiv * __builtin_amdgcn_rcp(G[i * gs + i]) : 0.0;
            double emax = e, emin = kept ? e : __builtin_inf();
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) {
                emax = fmax(emax, __shfl_xor(emax, off, 64));
                emin = fmin(emin, __shfl_xor(emin, off, 64));
            }
            if (l == 0) {
                ldouble* st = lp(st_);
                st[0] = (double)__builtin_popcount(dm & (live >= 16 ? 0xffffu : (1u << live) - 1u));
                st[1] = emax;
                st[2] = emin == __builtin_inf() ? 0.0 : emin;
            }
        }
    }
    if (sync) __syncthreads();
}

// G = X^T X over the first 4 KS rows of X (row stride XS), 16 x 16 row-major
// (stride XS) into Gout.  Wave w takes the k-steps w, w + 4, ...; its loads are
// all issued before its matrix-core chain; the four partial tiles are summed
// in wave order.  scr: 4 x 256 doubles.
__device__ __forceinline__ void gram16(const double* X_, int KS, double* scr_, double* Gout_) {
    const ldouble* X = lp(X_);
    ldouble* scr = lp(scr_);
    ldouble* Gout = lp(Gout_);
    const int tid = threadIdx.x, l = tid & 63, w = wave_id();
    constexpr int U = KMAX / 4;
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int ks = w + 4 * u;
        x[u] = ks < KS ? X[(4 * ks + (l >> 4)) * XS + (l & 15)] : 0.0;
    }
    d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < U; u += 2) {
        if (w + 4 * u >= KS) break;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], x[u], acc, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u + 1], x[u + 1], acc2, 0, 0, 0);
    }
    acc += acc2;
#pragma unroll
    for (int v = 0; v < 4; ++v) scr[w * 256 + ((l >> 4) + 4 * v) * 16 + (l & 15)] = acc[v];
    __syncthreads();
    Gout[(tid >> 4) * XS + (tid & 15)] = ((scr[tid] + scr[256 + tid]) + scr[512 + tid]) + scr[768 + tid];
    __syncthreads();
}

// X <- X T for the ntiles row tiles of X (row stride XS; T 16 x 16, row
// stride XS), in place: wave w takes the tiles w, w + 4, ..., reads all of
// them, then writes them.
__device__ __forceinline__ void xmul16(double* X_, int ntiles, const double* T_) {
    ldouble* X = lp(X_);
    const ldouble* T = lp(T_);
    const int tid = threadIdx.x, l = tid & 63, w = wave_id();
    constexpr int U = TMAX / 4;
    double bv[4], av[U][4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) bv[ks] = T[(4 * ks + (l >> 4)) * XS + (l & 15)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int t = w + 4 * u;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) av[u][ks] = t < ntiles ? X[(16 * t + (l & 15)) * XS + 4 * ks + (l >> 4)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int t = w + 4 * u;
        if (t >= ntiles) break;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][ks], bv[ks], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) X[(16 * t + (l >> 4) + 4 * v) * XS + (l & 15)] = acc[v];
    }
    __syncthreads();
}

}  // namespace

}  // namespace ircur
