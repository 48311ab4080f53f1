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
    core_body<T, F, R>(a, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// ----------------------------------------------------------------- pass ---

template <typename T, typename F, int R, bool LIT>
__global__ __launch_bounds__((64 * PassWaves<T, R>::value)) void pass_kernel(PassArgs a) {
    if (a.st->stop) return;
    __shared__ F red[PassTree<T, F, R>::nred];
    __shared__ double redzd[PassTree<T, F, R>::nzd];
    __shared__ double gsh[288];
    // XCD-aware order: workgroups are dealt to the 8 XCDs in turn, so work item
    // w = xcd * per + slot gives each XCD a contiguous range of (side, column
    // tile, row block) items: neighbouring tiles, which share the cache lines at
    // their edges, and the row blocks of one tile meet in the same L2
    const int ns0 = a.side[0].nsplit > 1 ? a.side[0].nsplit : 1;
    const int ns1 = a.side[1].nsplit > 1 ? a.side[1].nsplit : 1;
    const int nb0 = a.side[0].nwg * ns0;
    const int nbt = nb0 + a.side[1].nwg * ns1;
    const int per = (int)(gridDim.x >> 3);
    const int b = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (b >= nbt) {
        if (b == nbt && a.gapT) gap_estimate(a.gapT, a.gapinfo, a.gapR, gsh);   // (a spare workgroup)
        return;
    }
    if (b < nb0) {
        side_body<T, F, R, LIT>(a.side[0], b / ns0, b % ns0, a.zeta, a.zeta_f, red, redzd);
    } else {
        const int bb = b - nb0;
        side_body<T, F, R, LIT>(a.side[1], bb / ns1, bb % ns1, a.zeta, a.zeta_f, red, redzd);
    }
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
static hipError_t pass_r(const PassArgs& a, hipStream_t s) {
    const unsigned nb = (unsigned)(a.side[0].nwg * std::max(1, a.side[0].nsplit) +
                                   a.side[1].nwg * std::max(1, a.side[1].nsplit)) + (a.gapT ? 1 : 0);
    const unsigned grid = (nb + 7) / 8 * 8;          // a whole number of rounds over the 8 XCDs
    if (a.err_mode == 0) pass_kernel<T, F, R, true><<<grid, 64 * PassWaves<T, R>::value, 0, s>>>(a);
    else pass_kernel<T, F, R, false><<<grid, 64 * PassWaves<T, R>::value, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_core(const CoreArgs& a, int dtype, int R, hipStream_t s) {
    if (dtype == 0) { IRCUR_RANK_SWITCH(core_r, double, double, R, a, s) }
    if (dtype == 1) { IRCUR_RANK_SWITCH(core_r, float, float, R, a, s) }
    if (dtype == 2) { IRCUR_RANK_SWITCH(core_r, bf16_t, float, R, a, s) }
    return hipErrorInvalidValue;
}

hipError_t launch_pass(const PassArgs& a, int dtype, int R, hipStream_t s) {
    if (a.side[0].tiled && a.side[1].tiled) return launch_pass16(a, dtype, R, s);
    if (dtype == 0) { IRCUR_RANK_SWITCH(pass_r, double, double, R, a, s) }
    if (dtype == 1) { IRCUR_RANK_SWITCH(pass_r, float, float, R, a, s) }
    if (dtype == 2) { IRCUR_RANK_SWITCH(pass_r, bf16_t, float, R, a, s) }
    return hipErrorInvalidValue;
}

template <typename T, typename F, int R>
static int nsplit_r(int s, int tiles) {
    // blocks of about kPassSplitRows rows, at most 2048 workgroups per side
    int ns = (s + kPassSplitRows - 1) / kPassSplitRows;
    ns = std::min(ns, std::max(1, 2048 / std::max(tiles, 1)));
    ns = std::min(ns, kPassMaxSplit);
    return std::max(ns, 1);
}

int pass_nsplit(int dtype, int R, int s, int tiles) {
    if (dtype == 0) { IRCUR_RANK_SWITCH(nsplit_r, double, double, R, s, tiles) }
    if (dtype == 1) { IRCUR_RANK_SWITCH(nsplit_r, float, float, R, s, tiles) }
    if (dtype == 2) { IRCUR_RANK_SWITCH(nsplit_r, bf16_t, float, R, s, tiles) }
    return 1;
}

int pass_cols(int dtype, int R, bool matrix_core) {
    (void)R;
    if (matrix_core) return 32;
    return 64 * (dtype == 2 ? ColsPerLane<bf16_t>::value : (dtype == 1 ? ColsPerLane<float>::value
                                                                       : ColsPerLane<double>::value));
}

size_t pass_split_bytes(int dtype, int R) {
    const size_t f = dtype == 0 ? sizeof(double) : sizeof(float);
    const size_t V = pass_cols(dtype, R, false) / 64;
    return (size_t)R * V * 64 * f + 128 * sizeof(double);
}

hipError_t launch_finalize(const FinArgs& a, hipStream_t s) {
    finalize_kernel<<<1, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace ircur
