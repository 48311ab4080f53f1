// Outputs of Algorithm 1 outside the iteration loop:
//
//   export  C_k = [D - S_k]_{:,J}, R_k = [D - S_k]_{I,:} (eq. (2)), the sparse
//           blocks [S_k]_{I,:}, [S_k]_{:,J} (Phase I, eq. (4)) and U_k^+
//           (section 3.1), recomputed for the last completed iteration from
//           its input factors, index sets and threshold;
//   sparse  the full sparse part T_zeta(D - A_k B_k) over all of D (the
//           foreground of the video application, section 4.2).
//
// Every entry uses the same fma chain and threshold test as the iteration's
// core and pass kernels, so the exported blocks equal, bit for bit, the
// blocks the iteration used.
#include "ircur_device.h"

#include <stdint.h>

namespace ircur {

namespace {

// R_k and [S_k]_{I,:}: block (x, y) covers 256 columns of sampled row y.
template <typename T, typename F, int R>
__global__ __launch_bounds__(256) void cur_rows_kernel(CurArgs a) {
    const int ai = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= a.n2) return;
    const int64_t i = a.I[ai];
    const T* __restrict__ D = (const T*)a.D;
    const F* __restrict__ At = (const F*)a.At;
    const F* __restrict__ B = (const F*)a.B;
    const F d = ld<T, F>(D + i * a.ldD + j);
    F dot = F(0);
#pragma unroll
    for (int c = 0; c < R; ++c) dot = fmaT(At[c * a.n1 + i], B[c * a.n2 + j], dot);
    bool o;
    const F v = entry_value<F>(d, dot, a.zeta, a.zeta_f, &o);
    const int64_t e = (int64_t)ai * a.n2 + j;
    if (a.Rout) ((F*)a.Rout)[e] = v;
    if (a.SI) ((F*)a.SI)[e] = o ? d - dot : F(0);
}

// C_k and [S_k]_{:,J}: block (x, y) covers 256 rows of sampled column y,
// read as a contiguous row of D^T.
template <typename T, typename F, int R>
__global__ __launch_bounds__(256) void cur_cols_kernel(CurArgs a) {
    const int bj = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n1) return;
    const int64_t j = a.J[bj];
    const T* __restrict__ Dt = (const T*)a.Dt;
    const F* __restrict__ At = (const F*)a.At;
    const F* __restrict__ B = (const F*)a.B;
    const F d = ld<T, F>(Dt + j * a.ldDt + i);
    F dot = F(0);
#pragma unroll
    for (int c = 0; c < R; ++c) dot = fmaT(At[c * a.n1 + i], B[c * a.n2 + j], dot);
    bool o;
    const F v = entry_value<F>(d, dot, a.zeta, a.zeta_f, &o);
    const int64_t e = i * a.sJ + bj;
    if (a.Cout) ((F*)a.Cout)[e] = v;
    if (a.SJ) ((F*)a.SJ)[e] = o ? d - dot : F(0);
}

// U^+ = Q Ly^-T Wt^T (sJ x sI), in double, stored in the factor dtype.
template <typename F>
__global__ __launch_bounds__(256) void upinv_kernel(const double* __restrict__ V, const double* __restrict__ TA,
                                                    const double* __restrict__ W, int sI, int sJ, int R,
                                                    F* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)sI * sJ) return;
    const int j = (int)(e / sI), i = (int)(e - (int64_t)j * sI);
    double s = 0.0;
    for (int c = 0; c < R; ++c) {
        double t = 0.0;
        for (int d = 0; d < R; ++d) t = __builtin_fma(TA[c * R + d], W[(int64_t)i * R + d], t);
        s = __builtin_fma(V[(int64_t)j * R + c], t, s);
    }
    out[e] = (F)s;
}

// Full sparse part.  Block b covers 256 columns (column block b % ncb) of a
// band of kSparseRows rows (band b / ncb); the columns' factor entries stay
// in registers while the band streams through, kSparseU rows in flight.
constexpr int kSparseRows = 64;
constexpr int kSparseU = 4;

template <typename T, typename F, int R>
__global__ __launch_bounds__(256) void sparse_full_kernel(SparseArgs a, int64_t ncb) {
    const int64_t cb = blockIdx.x % ncb, band = blockIdx.x / ncb;
    const int64_t j = cb * 256 + threadIdx.x;
    const bool valid = j < a.n2;
    const int64_t jj = valid ? j : 0;
    const T* __restrict__ D = (const T*)a.D;
    const F* __restrict__ At = (const F*)a.At;
    const F* __restrict__ B = (const F*)a.B;
    T* __restrict__ S = (T*)a.S;
    F p[R];
#pragma unroll
    for (int c = 0; c < R; ++c) p[c] = B[c * a.n2 + jj];
    const int64_t i0 = band * kSparseRows;
    const int64_t i1 = i0 + kSparseRows < a.n1 ? i0 + kSparseRows : a.n1;
    uint32_t cnt = 0;
    for (int64_t ib = i0; ib < i1; ib += kSparseU) {
        F dv[kSparseU];
#pragma unroll
        for (int u = 0; u < kSparseU; ++u) {
            const int64_t i = ib + u < i1 ? ib + u : i1 - 1;
            dv[u] = ld<T, F>(D + i * a.ldD + jj);
        }
#pragma unroll
        for (int u = 0; u < kSparseU; ++u) {
            const int64_t i = ib + u;
            if (i < i1) {
                F dot = F(0);
#pragma unroll
                for (int c = 0; c < R; ++c) dot = fmaT(At[c * a.n1 + i], p[c], dot);
                const F x = dv[u] - dot;
                const bool o = above(x < F(0) ? -x : x, a.zeta, a.zeta_f);
                cnt += (o && valid) ? 1u : 0u;
                if (valid) S[i * a.ldS + j] = from_f<T>(o ? (double)x : 0.0);
            }
        }
    }
    if (a.nnz) {
        for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
        if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(a.nnz, (unsigned long long)cnt);
    }
}

template <typename T, typename F, int R>
hipError_t cur_r(const CurArgs& a, hipStream_t s) {
    if (a.Rout || a.SI) {
        dim3 g((unsigned)((a.n2 + 255) / 256), (unsigned)a.sI);
        cur_rows_kernel<T, F, R><<<g, 256, 0, s>>>(a);
    }
    if (a.Cout || a.SJ) {
        dim3 g((unsigned)((a.n1 + 255) / 256), (unsigned)a.sJ);
        cur_cols_kernel<T, F, R><<<g, 256, 0, s>>>(a);
    }
    return hipGetLastError();
}

template <typename T, typename F, int R>
hipError_t sparse_r(const SparseArgs& a, hipStream_t s) {
    const int64_t ncb = (a.n2 + 255) / 256, nb = (a.n1 + kSparseRows - 1) / kSparseRows;
    if (ncb * nb > 0x7fffffffLL) return hipErrorInvalidValue;
    sparse_full_kernel<T, F, R><<<(unsigned)(ncb * nb), 256, 0, s>>>(a, ncb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cur(const CurArgs& a, int dtype, int R, hipStream_t s) {
    if (a.sI > 65535 || a.sJ > 65535) return hipErrorInvalidValue;
    if (dtype == 0) { IRCUR_RANK_SWITCH(cur_r, double, double, R, a, s) }
    if (dtype == 1) { IRCUR_RANK_SWITCH(cur_r, float, float, R, a, s) }
    if (dtype == 2) { IRCUR_RANK_SWITCH(cur_r, bf16_t, float, R, a, s) }
    return hipErrorInvalidValue;
}

hipError_t launch_upinv(const double* V, const double* TA, const double* W, int sI, int sJ, int R,
                        void* out, int dtype, hipStream_t s) {
    const int64_t total = (int64_t)sI * sJ;
    const unsigned g = (unsigned)((total + 255) / 256);
    if (dtype == 0) upinv_kernel<double><<<g, 256, 0, s>>>(V, TA, W, sI, sJ, R, (double*)out);
    else upinv_kernel<float><<<g, 256, 0, s>>>(V, TA, W, sI, sJ, R, (float*)out);
    return hipGetLastError();
}

hipError_t launch_sparse_full(const SparseArgs& a, int dtype, int R, hipStream_t s) {
    if (dtype == 0) { IRCUR_RANK_SWITCH(sparse_r, double, double, R, a, s) }
    if (dtype == 1) { IRCUR_RANK_SWITCH(sparse_r, float, float, R, a, s) }
    if (dtype == 2) { IRCUR_RANK_SWITCH(sparse_r, bf16_t, float, R, a, s) }
    return hipErrorInvalidValue;
}

}  // namespace ircur
