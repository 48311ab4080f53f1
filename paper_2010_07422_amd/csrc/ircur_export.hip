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

// Full sparse part, vector form, for rows of D and S that start on lane-
// vector boundaries: a lane covers VEC consecutive columns (one 16- or 8-byte
// load and one store of that size per row), a wave a strip of 64 VEC columns,
// a workgroup a band of kSpBand rows of one strip (the four waves take
// kSpBand / 4 rows each, kSpU rows of loads in flight and the next kSpU
// requested while the current ones are processed).  The band's factor rows
// A_k[i, :] are staged in LDS; the lane's factor columns B_k[:, j] stay in
// registers.  D is read and S written with non-temporal hints (each byte is
// touched once).  Same fma chain and threshold test as every other kernel.
// (Measured on MI355X: bands of 256 rows with 8 rows in flight beat 128 / 8,
// 512 / 4, 512 / 8 and 256 / 16 on the 76800 x 1200 FP32 instance.)
#ifndef IRCUR_SP_BAND
#define IRCUR_SP_BAND 256
#endif
#ifndef IRCUR_SP_U
#define IRCUR_SP_U 8
#endif
constexpr int kSpBand = IRCUR_SP_BAND;
constexpr int kSpU = IRCUR_SP_U;

// Lane vector of the sparse kernel: NW 32-bit words (16 or 8 bytes) holding
// VEC elements of T.  16-byte vectors unless the lane's factor columns
// (R x VEC values in registers) would crowd out the rows in flight.
template <typename T, int R> struct SpLane {
    static constexpr int NW = (R * 16 / (int)sizeof(T) <= 48) ? 4 : 2;
    static constexpr int VEC = NW * 4 / (int)sizeof(T);
    typedef uint32_t W __attribute__((ext_vector_type(NW)));
};
template <typename T, typename F, int NW> struct SpPack;
template <int NW> struct SpPack<double, double, NW> {
    template <typename W> __device__ static void unpack(const W& w, double* o) {
#pragma unroll
        for (int k = 0; k < NW / 2; ++k) o[k] = __builtin_bit_cast(double, ((uint64_t)w[2 * k + 1] << 32) | w[2 * k]);
    }
    template <typename W> __device__ static W pack(const double* v) {
        W w;
#pragma unroll
        for (int k = 0; k < NW / 2; ++k) {
            const uint64_t u = __builtin_bit_cast(uint64_t, v[k]);
            w[2 * k] = (uint32_t)u;
            w[2 * k + 1] = (uint32_t)(u >> 32);
        }
        return w;
    }
};
template <int NW> struct SpPack<float, float, NW> {
    template <typename W> __device__ static void unpack(const W& w, float* o) {
#pragma unroll
        for (int k = 0; k < NW; ++k) o[k] = __uint_as_float(w[k]);
    }
    template <typename W> __device__ static W pack(const double* v) {
        W w;
#pragma unroll
        for (int k = 0; k < NW; ++k) w[k] = __float_as_uint((float)v[k]);
        return w;
    }
};
template <int NW> struct SpPack<bf16_t, float, NW> {
    template <typename W> __device__ static void unpack(const W& w, float* o) {
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            o[2 * k] = __uint_as_float(w[k] << 16);
            o[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
        }
    }
    template <typename W> __device__ static W pack(const double* v) {
        W w;
#pragma unroll
        for (int k = 0; k < NW; ++k)
            w[k] = (uint32_t)from_f<bf16_t>(v[2 * k]).bits | ((uint32_t)from_f<bf16_t>(v[2 * k + 1]).bits << 16);
        return w;
    }
};

template <typename T, typename F, int R>
__global__ __launch_bounds__(256) void sparse_vec_kernel(SparseArgs a, int64_t nstrip) {
    typedef SpLane<T, R> LN;
    typedef typename LN::W W;
    typedef SpPack<T, F, LN::NW> SV;
    constexpr int VEC = LN::VEC;
    constexpr int RW = kSpBand / 4;                     // rows per wave
    __shared__ F Ab[kSpBand * R];                       // Ab[i * R + c] = A_k[i0 + i, c]
    const int64_t strip = blockIdx.x % nstrip, band = blockIdx.x / nstrip;
    const int64_t i0 = band * kSpBand;
    const int nrow = (int)(a.n1 - i0 < kSpBand ? a.n1 - i0 : kSpBand);
    const F* __restrict__ At = (const F*)a.At;
    const F* __restrict__ B = (const F*)a.B;
    for (int e = threadIdx.x; e < kSpBand * R; e += 256) {
        const int c = e / kSpBand, ii = e - c * kSpBand;    // read along the rows of A_k^T
        Ab[ii * R + c] = ii < nrow ? At[c * a.n1 + i0 + ii] : F(0);
    }
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t j0 = (strip * 64 + lane) * VEC;
    int nv = (int)(a.n2 - j0 < VEC ? a.n2 - j0 : VEC);
    if (nv < 0) nv = 0;
    const int64_t jc = nv > 0 ? j0 : 0;                 // a lane past the last column reads column 0
    F p[R][VEC];
#pragma unroll
    for (int c = 0; c < R; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) p[c][v] = v < nv ? B[c * a.n2 + j0 + v] : F(0);
    const T* __restrict__ D = (const T*)a.D;
    T* __restrict__ S = (T*)a.S;
    const int r0 = wave * RW;
    const int r1 = nrow < r0 + RW ? nrow : r0 + RW;
    uint32_t cnt = 0;
    __syncthreads();
    if (r1 > r0) {
        auto load = [&](int ib, W* w) {
#pragma unroll
            for (int u = 0; u < kSpU; ++u) {
                const int row = ib + u < r1 ? ib + u : r1 - 1;
                const T* src = D + (i0 + row) * a.ldD + jc;
                if (nv == VEC) {
                    w[u] = __builtin_nontemporal_load((const W*)src);
                } else {
                    T tmp[VEC];
#pragma unroll
                    for (int v = 0; v < VEC; ++v) tmp[v] = v < nv ? src[v] : src[0];
                    w[u] = __builtin_bit_cast(W, tmp);
                }
            }
        };
        W nx[kSpU];
        load(r0, nx);
        for (int ib = r0; ib < r1; ib += kSpU) {
            W cur[kSpU];
#pragma unroll
            for (int u = 0; u < kSpU; ++u) cur[u] = nx[u];
            if (ib + kSpU < r1) load(ib + kSpU, nx);
#pragma unroll
            for (int u = 0; u < kSpU; ++u) {
                const int row = ib + u;
                if (row < r1) {
                    F d[VEC];
                    SV::unpack(cur[u], d);
                    const F* q = Ab + row * R;
                    double sv[VEC];
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        F dot = F(0);
#pragma unroll
                        for (int c = 0; c < R; ++c) dot = fmaT(q[c], p[c][v], dot);
                        const F x = d[v] - dot;
                        const bool o = above(x < F(0) ? -x : x, a.zeta, a.zeta_f);
                        cnt += (o && v < nv) ? 1u : 0u;
                        sv[v] = o ? (double)x : 0.0;
                    }
                    T* dst = S + (i0 + row) * a.ldS + j0;
                    if (nv == VEC) {
                        __builtin_nontemporal_store(SV::template pack<W>(sv), (W*)dst);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v)
                            if (v < nv) dst[v] = from_f<T>(sv[v]);
                    }
                }
            }
        }
    }
    if (a.nnz) {
        for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
        if (lane == 0 && cnt) atomicAdd(a.nnz, (unsigned long long)cnt);
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
    constexpr int VEC = SpLane<T, R>::VEC;
    constexpr int LB = SpLane<T, R>::NW * 4;       // bytes per lane and row
    const bool aligned = ((uintptr_t)a.D % LB) == 0 && ((uintptr_t)a.S % LB) == 0 &&
                         (a.ldD * (int64_t)sizeof(T)) % LB == 0 && (a.ldS * (int64_t)sizeof(T)) % LB == 0;
    if (aligned && R * VEC <= 96) {
        const int64_t nstrip = (a.n2 + 64 * VEC - 1) / (64 * VEC), nband = (a.n1 + kSpBand - 1) / kSpBand;
        if (nstrip * nband > 0x7fffffffLL) return hipErrorInvalidValue;
        sparse_vec_kernel<T, F, R><<<(unsigned)(nstrip * nband), 256, 0, s>>>(a, nstrip);
        return hipGetLastError();
    }
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
