// IRCUR streaming kernels for gfx950: transpose, core gather/threshold, the
// fused row/column pass and the end-of-iteration reduction.
//
// Notation (Algorithm 1): L_k = A_k B_k with A_k^T (R x n1) and B_k (R x n2)
// kept in HBM; I, J the sampled rows/columns; zeta = zeta_{k+1}.
//
//   core:  M = [D - S_{k+1}]_{I,J} where S_{k+1} = T_zeta[D - L_k] (eq. (4), (5))
//   pass:  row side   R = [D - S_{k+1}]_{I,:},  B_{k+1} = W_r^T R            (eq. (2), (3))
//          column side C = [D - S_{k+1}]_{:,J}, A_{k+1} = C V_r Sigma_r^+
//          plus the partial sums of the stopping criterion (eq. (6)).
//
// The pass works with the small quantity xr = v - (L_k)_ij, which is x where
// the entry is kept and 0 where it is thresholded (up to rounding), so that
// both the new factor and the residual of eq. (6) are formed without
// cancellation:
//   row side   g_j = W_r^T xr[:, j],  B_{k+1}[:, j] = Gamma B_k[:, j] + g_j,
//              Gamma = W_r^T A_k[I, :]  (so W_r^T R = Gamma B_k + g);
//              z = xr + Delta_a . B_k[:, j],  Delta = (I - W_r W_r^T) A_k[I, :],
//              so z = R - W_r Gamma B_k[:, j] and
//              ||R[:, j] - W_r B_{k+1}[:, j]||^2 = ||z||^2 - ||g_j||^2;
//   column side is the same with (A_k^T, J, Q, Gamma' = B_k[:, J] Q) and the
//   output row mapped by Ly^-T (A_{k+1} = C Q Ly^-T).
//   final: e_{k+1} and the device-side stop flag.
//
// Every element of a sampled row or column is computed as
//     x = d - sum_c q_c p_c       (one fma chain, c = 0 .. R-1, from 0)
//     v = |x| > zeta ? d - x : d  (entry of D - S_{k+1})
// with the same chain in the core kernel and in both sides of the pass, so
// the I x J block is bit-identical wherever it is computed.
#include "ircur_device.h"

#include <stdint.h>

#include <algorithm>

namespace ircur {

// ------------------------------------------------------------ transpose ---

template <typename E>
__global__ __launch_bounds__(256) void transpose_kernel(const E* __restrict__ src, int64_t lds,
                                                        E* __restrict__ dst, int64_t ldd,
                                                        int64_t rows, int64_t cols) {
    __shared__ E tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) tile[i][tx] = src[r * lds + c];
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int64_t c = c0 + i, r = r0 + tx;   // dst row c, column r
        if (c < cols && r < rows) dst[c * ldd + r] = tile[tx][i];
    }
}

hipError_t launch_transpose(const void* src, int64_t lds, void* dst, int64_t ldd,
                            int64_t rows, int64_t cols, int elem_bytes, hipStream_t s) {
    dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
    switch (elem_bytes) {
        case 2: transpose_kernel<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)src, lds, (uint16_t*)dst, ldd, rows, cols); break;
        case 4: transpose_kernel<uint32_t><<<grid, 256, 0, s>>>((const uint32_t*)src, lds, (uint32_t*)dst, ldd, rows, cols); break;
        case 8: transpose_kernel<uint64_t><<<grid, 256, 0, s>>>((const uint64_t*)src, lds, (uint64_t*)dst, ldd, rows, cols); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------- core ---

template <typename T, typename F, int R>
__global__ __launch_bounds__(256) void core_kernel(CoreArgs a) {
    if (a.st->stop) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.st->bar_ctr = 0u;  // for the SVD's grid barrier
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)a.sI * a.sJ) return;
    const int ai = (int)(idx / a.sJ), bj = (int)(idx - (int64_t)ai * a.sJ);
    const int64_t i = a.I[ai], j = a.J[bj];
    const T* __restrict__ D = (const T*)a.D;
    const F* __restrict__ At = (const F*)a.At;
    const F* __restrict__ B = (const F*)a.B;
    const F d = ld<T, F>(D + i * a.ldD + j);
    F dot = F(0);
#pragma unroll
    for (int c = 0; c < R; ++c) dot = fmaT(At[c * a.n1 + i], B[c * a.n2 + j], dot);
    bool o;
    const F v = entry_value<F>(d, dot, a.zeta, a.zeta_f, &o);
    const double mv = (double)v;
    a.M[idx] = mv;
    const int sJ16 = ((a.sJ + 15) / 16) * 16, sI16 = ((a.sI + 15) / 16) * 16;
    a.MA[((size_t)(ai >> 4) * (sJ16 >> 2) + (bj >> 2)) * 64 + ((bj & 3) << 4) + (ai & 15)] = mv;
    a.MB[((size_t)(bj >> 4) * (sI16 >> 2) + (ai >> 2)) * 64 + ((ai & 3) << 4) + (bj & 15)] = mv;
}

// ----------------------------------------------------------------- pass ---

// One workgroup: 64 consecutive outputs (one per lane) x all s gathered rows.
// Wave w takes a contiguous quarter of the rows and keeps U row loads of D in
// flight (the next group is issued before the current one is consumed); the
// four partial sums are reduced in LDS at the end.  The per-row data
// (gathered factor row, projection row, Delta row; QS elements per row, 16-byte
// aligned) is wave-uniform: the workgroup stages it in LDS with batched
// 16-byte loads (all rows at once unless they exceed the LDS budget) and reads
// it back as broadcast loads.  The index arrays carry kIndexPad valid trailing
// entries, so a group may read past the end of a wave's rows.
template <typename T> struct RowsInFlight { static constexpr int value = 8; };
template <> struct RowsInFlight<bf16_t> { static constexpr int value = 16; };
template <> struct RowsInFlight<double> { static constexpr int value = 4; };

template <typename T, typename F, int R, bool LIT>
__device__ __forceinline__ void side_body(const SideArgs& S, int wg, double zeta, float zeta_f,
                                          F (*red)[R][64], double (*redz)[64], double (*redd)[64],
                                          F* qstage, int segmax) {
    constexpr int U = RowsInFlight<T>::value;
    constexpr int QS = RowStride<F, R>::value;
    constexpr int UPR = QS * (int)sizeof(F) / 16;          // 16-byte units per row
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t col = (int64_t)wg * 64 + lane;
    const bool valid = col < S.n;
    const int64_t n = S.n;
    const T* __restrict__ X = (const T*)S.X;
    const F* __restrict__ P = (const F*)S.P;
    const uint4* __restrict__ rd4 = (const uint4*)S.rowdata;
    const int32_t* __restrict__ rows = S.rows;
    const int64_t ldX = S.ldX;

    F p[R];
#pragma unroll
    for (int c = 0; c < R; ++c) p[c] = valid ? P[c * n + col] : F(0);
    F acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = F(0);
    F zz = F(0), dd = F(0);
    const T* __restrict__ Xc = X + (valid ? col : 0);   // invalid lanes read column 0
    const int chunk = (S.s + 3) >> 2;
    const int a_begin = wave * chunk;
    const int a_end = min(S.s, a_begin + chunk);
    // rows per stage: whole chunk if it fits, else segmax (a multiple of U)
    const int SEG = chunk <= segmax ? ((chunk + U - 1) / U) * U : segmax;
    F* __restrict__ qw = qstage + wave * (SEG * QS);

    F dv[U];
    if (a_end > a_begin) {
#pragma unroll
        for (int u = 0; u < U; ++u) dv[u] = ld<T, F>(Xc + (int64_t)rows[a_begin + u] * ldX);
    }
    for (int seg0 = 0; seg0 < chunk; seg0 += SEG) {       // uniform over the workgroup
        const int sb = a_begin + seg0;
        const int se = min(a_end, sb + SEG);
        __syncthreads();                                  // previous segment consumed
        {
            const int units = 4 * SEG * UPR;
            for (int base = threadIdx.x; base < units; base += 256 * 8) {
                uint4 v[8];
                int dst[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int un = base + u * 256;
                    dst[u] = -1;
                    if (un < units) {
                        const int w = un / (SEG * UPR);
                        const int rem = un - w * (SEG * UPR);
                        const int rr = rem / UPR, kk = rem - rr * UPR;
                        const int row = w * chunk + seg0 + rr;
                        if (seg0 + rr < chunk && row < S.s) {
                            v[u] = rd4[(int64_t)row * UPR + kk];
                            dst[u] = un;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (dst[u] >= 0) ((uint4*)qstage)[dst[u]] = v[u];
            }
        }
        __syncthreads();
        for (int a0 = sb; a0 < se; a0 += U) {
            F cur[U];
#pragma unroll
            for (int u = 0; u < U; ++u) cur[u] = dv[u];
            if (a0 + U < a_end) {
#pragma unroll
                for (int u = 0; u < U; ++u) dv[u] = ld<T, F>(Xc + (int64_t)rows[a0 + U + u] * ldX);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int a = a0 + u;
                if (a < se) {
                    const F d = valid ? cur[u] : F(0);
                    const F* q = qw + (a - sb) * QS;
                    F dot = F(0);
#pragma unroll
                    for (int c = 0; c < R; ++c) dot = fmaT(q[c], p[c], dot);
                    const F x = d - dot;
                    const F xr = above(x < F(0) ? -x : x, zeta, zeta_f) ? F(0) : x;
#pragma unroll
                    for (int c = 0; c < R; ++c) acc[c] = fmaT(q[R + c], xr, acc[c]);
                    if (LIT) {
                        F z = xr;
#pragma unroll
                        for (int c = 0; c < R; ++c) z = fmaT(q[2 * R + c], p[c], z);
                        zz = fmaT(z, z, zz);
                    } else {
                        zz = fmaT(xr, xr, zz);
                    }
                    dd = fmaT(d, d, dd);
                }
            }
        }
    }

#pragma unroll
    for (int c = 0; c < R; ++c) red[wave][c][lane] = acc[c];
    redz[wave][lane] = (double)zz;
    redd[wave][lane] = (double)dd;
    __syncthreads();
    if (wave == 0) {
        const F* __restrict__ Gm = (const F*)S.Gm;
        const F* __restrict__ Tm = (const F*)S.outmat;
        F* __restrict__ out = (F*)S.out;
        double corr = 0.0;
        F val[R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const F g = ((red[0][c][lane] + red[1][c][lane]) + red[2][c][lane]) + red[3][c][lane];
            if (LIT) corr = __builtin_fma((double)g, (double)g, corr);
            F base = F(0);
#pragma unroll
            for (int e = 0; e < R; ++e) base = fmaT(Gm[c * R + e], p[e], base);
            val[c] = base + g;
        }
#pragma unroll
        for (int c = 0; c < R; ++c) {
            F o = val[c];
            if (Tm) {
                o = F(0);
#pragma unroll
                for (int d = 0; d < R; ++d) o = fmaT(val[d], Tm[d * R + c], o);
            }
            if (valid) out[c * n + col] = o;
        }
        double zl = ((redz[0][lane] + redz[1][lane]) + redz[2][lane]) + redz[3][lane];
        double dl = ((redd[0][lane] + redd[1][lane]) + redd[2][lane]) + redd[3][lane];
        if (!valid) { zl = 0.0; dl = 0.0; corr = 0.0; }
        const double res = wave_sum(zl - corr);
        const double dsum = wave_sum(dl);
        if (lane == 0) {
            S.part[2 * wg] = res;
            S.part[2 * wg + 1] = dsum;
        }
    }
}

template <typename T, typename F, int R, bool LIT>
__global__ __launch_bounds__(256) void pass_kernel(PassArgs a) {
    if (a.st->stop) return;
    __shared__ F red[4][R][64];
    __shared__ double redz[4][64];
    __shared__ double redd[4][64];
    extern __shared__ __align__(16) unsigned char dyn[];
    F* qstage = (F*)dyn;
    const int wg = blockIdx.x;
    if (wg < a.side[0].nwg)
        side_body<T, F, R, LIT>(a.side[0], wg, a.zeta, a.zeta_f, red, redz, redd, qstage, a.segmax);
    else
        side_body<T, F, R, LIT>(a.side[1], wg - a.side[0].nwg, a.zeta, a.zeta_f, red, redz, redd, qstage,
                                a.segmax);
}

// ------------------------------------------------------------- finalize ---

__global__ __launch_bounds__(256) void finalize_kernel(FinArgs a) {
    if (a.st->stop) return;
    __shared__ double sh[4][256];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w = threadIdx.x; w < a.nrow; w += 256) {
        v[0] += a.part_row[2 * w];
        v[1] += a.part_row[2 * w + 1];
    }
    for (int w = threadIdx.x; w < a.ncol; w += 256) {
        v[2] += a.part_col[2 * w];
        v[3] += a.part_col[2 * w + 1];
    }
    for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double rr = sh[0][0], dr = sh[1][0], rc = sh[2][0], dc = sh[3][0];
        DevState* st = a.st;
        const bool finite = __builtin_isfinite(rr) && __builtin_isfinite(dr) &&
                            __builtin_isfinite(rc) && __builtin_isfinite(dc);
        double e;
        const double den = __builtin_sqrt(dr) + __builtin_sqrt(dc);
        if (!finite) {
            e = __builtin_nan("");
            st->nonfinite = 1;
        } else if (den == 0.0) {
            e = 0.0;
        } else {
            e = (__builtin_sqrt(rr > 0.0 ? rr : 0.0) + __builtin_sqrt(rc > 0.0 ? rc : 0.0)) / den;
        }
        a.hist[a.k] = e;
        st->e_last = e;
        st->k_done = a.k + 1;
        if (!finite || e <= a.eps || a.k + 1 >= a.max_iter || st->svd_fail) st->stop = 1;
    }
}

// ------------------------------------------------------------ launchers ---

template <typename T, typename F, int R>
static hipError_t core_r(const CoreArgs& a, hipStream_t s) {
    const int64_t total = (int64_t)a.sI * a.sJ;
    const unsigned grid = (unsigned)((total + 255) / 256);
    core_kernel<T, F, R><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <typename T, typename F, int R>
static hipError_t pass_r(const PassArgs& a0, hipStream_t s) {
    PassArgs a = a0;
    constexpr int U = RowsInFlight<T>::value;
    constexpr int rowbytes = RowStride<F, R>::value * (int)sizeof(F);
    int segmax = (kPassStageBytes / (4 * rowbytes)) / U * U;
    if (segmax < U) segmax = U;
    const int chunk = (std::max(a.side[0].s, a.side[1].s) + 3) / 4;
    const int seg = chunk <= segmax ? ((chunk + U - 1) / U) * U : segmax;
    a.segmax = segmax;
    const size_t lds = (size_t)4 * seg * rowbytes;
    static bool attr[2] = {false, false};
    const int li = a.err_mode == 0 ? 0 : 1;
    const void* fn = a.err_mode == 0 ? (const void*)pass_kernel<T, F, R, true> : (const void*)pass_kernel<T, F, R, false>;
    if (!attr[li]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kPassStageBytes);
        if (e != hipSuccess) return e;
        attr[li] = true;
    }
    const unsigned grid = (unsigned)(a.side[0].nwg + a.side[1].nwg);
    if (a.err_mode == 0) pass_kernel<T, F, R, true><<<grid, 256, lds, s>>>(a);
    else pass_kernel<T, F, R, false><<<grid, 256, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_core(const CoreArgs& a, int dtype, int R, hipStream_t s) {
    if (dtype == 0) { IRCUR_RANK_SWITCH(core_r, double, double, R, a, s) }
    if (dtype == 1) { IRCUR_RANK_SWITCH(core_r, float, float, R, a, s) }
    if (dtype == 2) { IRCUR_RANK_SWITCH(core_r, bf16_t, float, R, a, s) }
    return hipErrorInvalidValue;
}

hipError_t launch_pass(const PassArgs& a, int dtype, int R, hipStream_t s) {
    if (dtype == 0) { IRCUR_RANK_SWITCH(pass_r, double, double, R, a, s) }
    if (dtype == 1) { IRCUR_RANK_SWITCH(pass_r, float, float, R, a, s) }
    if (dtype == 2) { IRCUR_RANK_SWITCH(pass_r, bf16_t, float, R, a, s) }
    return hipErrorInvalidValue;
}

hipError_t launch_finalize(const FinArgs& a, hipStream_t s) {
    finalize_kernel<<<1, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace ircur
