// Device helpers shared by the IRCUR kernel files: element loads, the fma
// chain of an entry of L_k, the exact threshold test of eq. (4) and the
// rank dispatch.
#pragma once

#include "ircur_internal.h"
#include "ircur_gptr.h"

#include <algorithm>

namespace ircur {

// ---------------------------------------------------------------- types ---

struct bf16_t { uint16_t bits; };
// 16-byte vector (a native vector type, so arrays of it stay in registers)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T, typename F> __device__ __forceinline__ F ld(const T* p);
template <> __device__ __forceinline__ double ld<double, double>(const double* p) { return *p; }
template <> __device__ __forceinline__ float ld<float, float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float ld<bf16_t, float>(const bf16_t* p) {
    return __uint_as_float(((uint32_t)p->bits) << 16);
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// |x| > zeta evaluated exactly: in float, against the largest float <= zeta.
__device__ __forceinline__ bool above(double ax, double z, float) { return ax > z; }
__device__ __forceinline__ bool above(float ax, double, float zf) { return ax > zf; }

template <typename F>
__device__ __forceinline__ F entry_value(F d, F dot, double zeta, float zeta_f, bool* is_out) {
    const F x = d - dot;
    const bool o = above(x < F(0) ? -x : x, zeta, zeta_f);
    *is_out = o;
    return o ? d - x : d;
}

__device__ __forceinline__ double wave_sum(double v) {
    // Fixed butterfly over the 64 lanes: every lane ends with the same sum,
    // formed in the same order on every run.
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Gap estimate of the one-launch SVD, made by a spare workgroup of the pass
// launch that follows it: sigma_{r+1} / sigma_r ~ sqrt(bx / lambda_min(Gy_rr))
// with bx the extra columns' largest Rayleigh quotient (info->bx) and
// lambda_min(Gy_rr) = 1 / lambda_max(Ly^-T Ly^-1) (T = Ly^-T, R x R), by eight
// power steps on the first wave.  T and the vectors stay in LDS (sh: 288
// doubles), so that the pass kernels keep their register budget.
__device__ __forceinline__ void gap_estimate(const double* T, SvdInfo* info, int R, double* sh) {
    if (threadIdx.x >= 64) return;
    const int l = threadIdx.x;
    double* Ts = sh;                           // R x R
    double* vs = sh + 256;                     // 16
    double* ws = sh + 272;                     // 16
    for (int e = l; e < R * R; e += 64) Ts[e] = T[e];
    const double bx = info->bx;
    double gap = -1.0;
    if (bx >= 0.0) {
        double v = l < R ? 1.0 : 0.0, lam = 0.0;
        for (int s = 0; s < 8; ++s) {
            if (l < 16) vs[l] = v;
            __builtin_amdgcn_wave_barrier();
            double w = 0.0;
            if (l < R)
                for (int k = 0; k < R; ++k) w = __builtin_fma(Ts[k * R + l], vs[k], w);   // (T^T v)_l
            if (l < 16) ws[l] = w;
            __builtin_amdgcn_wave_barrier();
            double u = 0.0;
            if (l < R)
                for (int k = 0; k < R; ++k) u = __builtin_fma(Ts[l * R + k], ws[k], u);   // (T w)_l
            __builtin_amdgcn_wave_barrier();
            const double nv = __builtin_sqrt(wave_sum(u * u));
            const double vv = __builtin_sqrt(wave_sum(v * v));
            lam = vv > 0.0 ? nv / vv : 0.0;
            v = nv > 0.0 ? u / nv : 0.0;
        }
        gap = __builtin_sqrt(bx * lam);
    }
    if (l == 0) info->gap = gap;
}

// Round a float to the nearest bfloat16 (ties to even); NaN stays NaN.
__device__ __forceinline__ bf16_t to_bf16(float v) {
    uint32_t u = __float_as_uint(v);
    bf16_t b;
    if ((u & 0x7fffffffu) > 0x7f800000u) { b.bits = (uint16_t)((u >> 16) | 0x40u); return b; }
    u += 0x7fffu + ((u >> 16) & 1u);
    b.bits = (uint16_t)(u >> 16);
    return b;
}

template <typename T> __device__ __forceinline__ T from_f(double v);
template <> __device__ __forceinline__ double from_f<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_f<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ bf16_t from_f<bf16_t>(double v) { return to_bf16((float)v); }

// Gate of the unrolled mode: g = sigmoid((|x| - zeta) / tauz), tauz = tau_rel zeta
// (tends to the hard threshold of eq. (4) as tau_rel -> 0).
__device__ __forceinline__ double exp_t(double v) { return exp(v); }
__device__ __forceinline__ float exp_t(float v) { return expf(v); }
template <typename F>
__device__ __forceinline__ F gate_value(F x, F zeta, F tauz) {
    const F ax = x < F(0) ? -x : x;
    return F(1) / (F(1) + exp_t(-(ax - zeta) / tauz));
}

// The vector pass (padded ranks below 8 or above 16, and runs whose SVD takes
// several launches; ircur_pass16.hip has the matrix-core one).  One
// workgroup: 64 consecutive outputs (one column per lane) x a block of the s
// gathered rows (row split: the blocks of a column tile meet through a ticket,
// see side_body).  The NW waves split the block's rows into contiguous
// chunks; each keeps U row loads in flight.  The per-wave partial sums are
// combined by a fixed binary tree in LDS (the result does not depend on
// scheduling).  The per-row data (gathered factor row, projection row, Delta
// row; QS elements per row, 16-byte aligned) is wave-uniform: each wave reads
// it through the scalar cache into SGPRs, the FMAs' uniform operand.  The
// index arrays carry kIndexPad valid trailing entries, so a group may read
// past the end of a wave's rows.
// Rows in flight per wave (the next group is loaded while the current one is
// processed), columns per lane and waves per workgroup, by storage type.
// (Measured on MI355X at n = 10^4: FP64 is fastest with 8 waves, BF16 and
// FP32 with 4 waves and one column per lane; BF16 with 32 rows in flight,
// which covers a wave's share of a 128-row block in one group.)
template <typename T> struct RowsInFlight { static constexpr int value = 8; };
template <> struct RowsInFlight<bf16_t> { static constexpr int value = 32; };
template <> struct RowsInFlight<double> { static constexpr int value = 8; };
template <typename T> struct ColsPerLane { static constexpr int value = 1; };
template <typename T, int R> struct PassWaves { static constexpr int value = 4; };
template <int R> struct PassWaves<double, R> { static constexpr int value = 8; };

// Static LDS of the pass (bytes): one stage of the reduction tree.
template <typename T, typename F, int R> struct PassTree {
    static constexpr int V = ColsPerLane<T>::value;
    static constexpr int slots = PassWaves<T, R>::value / 2;
    static constexpr int nred = slots * R * 64 * V;          // F values
    static constexpr int nzd = slots * 64 * 2;               // doubles (zz, dd)
    static constexpr size_t bytes = (size_t)nred * sizeof(F) + (size_t)nzd * sizeof(double);
};

// Element loads of one row for the V columns of a lane.
template <typename T, typename F, int V>
__device__ __forceinline__ void load_row(const T* __restrict__ row, int64_t col0, int nvalid, bool vec, F* out) {
    if (V == 1) {
        out[0] = ld<T, F>(row + (nvalid > 0 ? col0 : 0));
    } else {
        if (vec && nvalid == V) {
            const uint32_t u = *(const uint32_t*)(row + col0);
            out[0] = __uint_as_float(u << 16);
            out[1] = __uint_as_float(u & 0xffff0000u);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) out[v] = ld<T, F>(row + (v < nvalid ? col0 + v : 0));
        }
    }
}

template <typename T, typename F, int R, bool LIT, bool GATE = false>
__device__ __forceinline__ void side_body(const SideArgs& S, int wg, int blk, double zeta, float zeta_f,
                                          F* red, double* redzd, F tauz = F(0)) {
    constexpr int NW = PassWaves<T, R>::value;
    constexpr int V = ColsPerLane<T>::value;
    constexpr int U = RowsInFlight<T>::value;
    static_assert(U <= kIndexPad, "the row read-ahead must stay inside the index padding");
    static_assert(V == 1 || sizeof(T) == 2, "two columns per lane only for 16-bit storage");
    constexpr int QS = RowStride<F, R>::value;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n = S.n;
    const int64_t col0 = ((int64_t)wg * 64 + lane) * V;
    int nvalid = (int)(n - col0);
    if (nvalid < 0) nvalid = 0;
    if (nvalid > V) nvalid = V;
    const T* __restrict__ X = (const T*)S.X;
    const F* __restrict__ P = (const F*)S.P;
    const int32_t* __restrict__ rows = S.rows;
    const int64_t ldX = S.ldX;
    const bool vec = (ldX % 2) == 0;                         // aligned pairs in every row

    F p[V][R];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int c = 0; c < R; ++c) p[v][c] = v < nvalid ? P[c * n + col0 + v] : F(0);
    F acc[V][R];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int c = 0; c < R; ++c) acc[v][c] = F(0);
    F zz = F(0), dd = F(0);
    // this workgroup's rows [rb, re): row block blk of the tile, split over the waves
    const int ns = S.nsplit > 1 ? S.nsplit : 1;
    const int bsz = (S.s + ns - 1) / ns;
    const int rb = min(S.s, blk * bsz);
    const int re = min(S.s, rb + bsz);
    const int chunk = (re - rb + NW - 1) / NW;
    const int a_begin = rb + wave * chunk;
    const int a_end = min(re, a_begin + chunk);
    // the per-row data (gathered factor row, projection row, Delta row) is the
    // same for every lane: it is read through the scalar cache into SGPRs,
    // which the FMAs take as their uniform operand
    typedef const __attribute__((address_space(4))) F* CF;
    typedef const __attribute__((address_space(4))) int32_t* CI;
    const CF rdc = (CF)S.rowdata;
    const CI rowc = (CI)S.rows;
    F nx[U][V];                                           // next group of rows (loaded ahead)
    // 32-bit factors: the next row's data is requested while the current row
    // is processed (scalar loads return in any order, so the wait for the
    // current row's data is placed before the next request); 64-bit factors
    // would need more SGPRs than a wave has for the two rows
    constexpr bool PF = sizeof(F) == 4;
    constexpr int NQ = LIT ? 3 * R : 2 * R;
    static_assert(!PF || U % 2 == 0, "the two row buffers alternate within a group");
    F qb[2][3 * R];                                       // rows of even / odd position in a group
    if (PF && a_end > a_begin) {
        const CF q = rdc + (size_t)a_begin * QS;
#pragma unroll
        for (int c = 0; c < NQ; ++c) qb[0][c] = q[c];
    }
    if (a_end > a_begin) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            load_row<T, F, V>(X + (int64_t)rowc[a_begin + u] * ldX, col0, nvalid, vec, nx[u]);
    }
    for (int a0 = a_begin; a0 < a_end; a0 += U) {
        F dv[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) dv[u][v] = nx[u][v];
        if (a0 + U < a_end) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                load_row<T, F, V>(X + (int64_t)rowc[a0 + U + u] * ldX, col0, nvalid, vec, nx[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int a = a0 + u;
            if (a < a_end) {
                    F* qa = qb[u & 1];
                    if (PF) {
                        __builtin_amdgcn_s_waitcnt(0xc07f);       // lgkmcnt(0): row a's data is here
                        __builtin_amdgcn_sched_barrier(0);
                        const CF q = rdc + (size_t)(a + 1 < a_end ? a + 1 : a) * QS;
#pragma unroll
                        for (int c = 0; c < NQ; ++c) qb[(u + 1) & 1][c] = q[c];
                        __builtin_amdgcn_sched_barrier(0);
                    } else {
                        const CF q = rdc + (size_t)a * QS;
#pragma unroll
                        for (int c = 0; c < NQ; ++c) qa[c] = q[c];
                    }
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const F d = v < nvalid ? dv[u][v] : F(0);
                        F dot = F(0);
#pragma unroll
                        for (int c = 0; c < R; ++c) dot = fmaT(qa[c], p[v][c], dot);
                        const F x = d - dot;
                        F xr;
                        if (GATE) xr = x - x * gate_value<F>(x, (F)zeta, tauz);
                        else xr = above(x < F(0) ? -x : x, zeta, zeta_f) ? F(0) : x;
#pragma unroll
                        for (int c = 0; c < R; ++c) acc[v][c] = fmaT(qa[R + c], xr, acc[v][c]);
                        if (LIT) {
                            F z = xr;
#pragma unroll
                            for (int c = 0; c < R; ++c) z = fmaT(qa[2 * R + c], p[v][c], z);
                            zz = fmaT(z, z, zz);
                        } else {
                            zz = fmaT(xr, xr, zz);
                        }
                        dd = fmaT(d, d, dd);
                    }
            }
        }
    }

    // fixed reduction tree over the waves: NW/2 -> ... -> 1
    double zl = (double)zz, dl = (double)dd;
#pragma unroll
    for (int half = NW / 2; half >= 1; half >>= 1) {
        __syncthreads();
        if (wave >= half && wave < 2 * half) {
            const int slot = wave - half;
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int c = 0; c < R; ++c) red[((slot * R + c) * V + v) * 64 + lane] = acc[v][c];
            redzd[(slot * 2) * 64 + lane] = zl;
            redzd[(slot * 2 + 1) * 64 + lane] = dl;
        }
        __syncthreads();
        if (wave < half) {
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int c = 0; c < R; ++c) acc[v][c] += red[((wave * R + c) * V + v) * 64 + lane];
            zl += redzd[(wave * 2) * 64 + lane];
            dl += redzd[(wave * 2 + 1) * 64 + lane];
        }
    }
    if (ns > 1) {
        // row-split tile: publish this block's sums (device-scope stores, complete
        // before the ticket is taken); the last block of the tile adds all blocks
        // in block order, so the result does not depend on the arrival order
        __shared__ int last_blk;
        if (wave == 0) {
            F* pa = (F*)S.pacc + (size_t)(wg * ns + blk) * (R * V * 64);
            double* pz = S.pzd + (size_t)(wg * ns + blk) * 128;
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int c = 0; c < R; ++c)
                    __hip_atomic_store(pa + (c * V + v) * 64 + lane, acc[v][c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(pz + lane, zl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(pz + 64 + lane, dl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
            if (lane == 0) {
                const uint32_t t = __hip_atomic_fetch_add(S.cnt + wg, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last_blk = t == (uint32_t)(ns - 1) ? 1 : 0;
            }
        }
        __syncthreads();
        if (!last_blk) return;
        if (wave == 0) {
            if (lane == 0) __hip_atomic_store(S.cnt + wg, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int c = 0; c < R; ++c) acc[v][c] = F(0);
            zl = 0.0;
            dl = 0.0;
            for (int b = 0; b < ns; ++b) {
                const F* pa = (const F*)S.pacc + (size_t)(wg * ns + b) * (R * V * 64);
                const double* pz = S.pzd + (size_t)(wg * ns + b) * 128;
#pragma unroll
                for (int v = 0; v < V; ++v)
#pragma unroll
                    for (int c = 0; c < R; ++c)
                        acc[v][c] += __hip_atomic_load(pa + (c * V + v) * 64 + lane, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                zl += __hip_atomic_load(pz + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                dl += __hip_atomic_load(pz + 64 + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (wave == 0) {
        const F* __restrict__ Gm = (const F*)S.Gm;
        const F* __restrict__ Tm = (const F*)S.outmat;
        F* __restrict__ out = (F*)S.out;
        double corr = 0.0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            F val[R];
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const F g = acc[v][c];
                if (LIT && v < nvalid) corr = __builtin_fma((double)g, (double)g, corr);
                F base = F(0);
#pragma unroll
                for (int e = 0; e < R; ++e) base = fmaT(Gm[c * R + e], p[v][e], base);
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
                if (v < nvalid) out[c * n + col0 + v] = o;
            }
        }
        if (nvalid == 0) { zl = 0.0; dl = 0.0; corr = 0.0; }
        const double res = wave_sum(zl - corr);
        const double dsum = wave_sum(dl);
        if (lane == 0) {
            S.part[2 * wg] = res;
            S.part[2 * wg + 1] = dsum;
        }
    }
}



// One element of the core M = [D - S_{k+1}]_{I,J} (eq. (4), (5)) at flat
// index idx = a * |J| + b, in every layout the SVD reads (see CoreArgs), and
// the compact factor copies.  Shared by the core kernel and the core launch
// of the one-launch SVD.
template <typename T, typename F, int R>
__device__ __forceinline__ void core_body(const CoreArgs& a, int64_t idx) {
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
    if (a.MB) a.MB[((size_t)(bj >> 4) * (sI16 >> 2) + (ai >> 2)) * 64 + ((ai & 3) << 4) + (bj & 15)] = mv;
    if (a.Abc && bj == 0) {
#pragma unroll
        for (int c = 0; c < R; ++c) a.Abc[(size_t)ai * 16 + c] = (double)At[c * a.n1 + i];
    }
    if (a.Bsc && ai == 0) {
#pragma unroll
        for (int c = 0; c < R; ++c) a.Bsc[(size_t)c * sJ16 + bj] = (double)B[c * a.n2 + j];
    }
}

#define IRCUR_RANK_SWITCH(FN, T, F, R, ...)                     \
    switch (R) {                                                \
        case 1: return FN<T, F, 1>(__VA_ARGS__);                \
        case 2: return FN<T, F, 2>(__VA_ARGS__);                \
        case 3: return FN<T, F, 3>(__VA_ARGS__);                \
        case 4: return FN<T, F, 4>(__VA_ARGS__);                \
        case 5: return FN<T, F, 5>(__VA_ARGS__);                \
        case 6: return FN<T, F, 6>(__VA_ARGS__);                \
        case 8: return FN<T, F, 8>(__VA_ARGS__);                \
        case 10: return FN<T, F, 10>(__VA_ARGS__);              \
        case 12: return FN<T, F, 12>(__VA_ARGS__);              \
        case 16: return FN<T, F, 16>(__VA_ARGS__);              \
        case 20: return FN<T, F, 20>(__VA_ARGS__);              \
        case 24: return FN<T, F, 24>(__VA_ARGS__);              \
        case 32: return FN<T, F, 32>(__VA_ARGS__);              \
        default: return hipErrorInvalidValue;                   \
    }


}  // namespace ircur
