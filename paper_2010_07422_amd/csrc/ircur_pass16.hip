// Fused row/column pass (section 3.2: the threshold T_zeta of eq. (4) on the
// sampled rows and columns, and the products that give the next factors,
// eq. (5)) on the matrix cores, for padded ranks 8 <= R <= 16.
//
// For one side (rows I of D, or rows J of D^T) and every column j:
//   x_aj  = D[rows_a, j] - sum_c q_a[c] P[c, j]         (the entry of D - L_k)
//   xr_aj = x_aj if |x_aj| <= zeta, else 0              (the entry of D - S_{k+1} - L_k)
//   acc[c, j] = sum_a w_a[c] xr_aj                      (projection of the residual)
//   z_aj  = xr_aj + sum_c t_a[c] P[c, j]                (the residual of the next iterate)
//   out[:, j] = Tm^T (Gm P[:, j] + acc[:, j])           (the next factor column)
// with the per-row data [q_a | w_a | t_a] written by the SVD (in the lane
// order of the operands below, one block of (2 ceil(R/4) + 4) x 64 values per
// 16-row tile, zero past the sampled rows), plus the sums
// of z^2 (minus |acc|^2) and of d^2 per column tile for the stopping test.
//
// A workgroup owns 32 columns (two column tiles) and every sampled row, so no
// partial sums leave it: each of its four waves takes one column tile and
// every other 16-row tile, a few tiles at a time with all their operands
// requested before the first product (all nine of its tiles at once with 32-bit
// arithmetic and at most 288 sampled rows; the sampled row indices are staged
// in LDS first).  On one tile, the
// 16 x 16 block of x is the accumulator of R-deep products q P
// (v_mfma_*_16x16x4); the thresholded block stays in those registers and is
// the B operand of the products w^T xr that accumulate acc (the four rows a
// lane holds are one k-step of those products: the rows of the k-steps are
// taken in the order of the accumulator layout, which only reorders a sum),
// and the starting value of the products t P that give z.  The waves' acc
// and sums meet in LDS in wave order; the output map is two more
// products.  Work items are dealt so that each XCD takes a contiguous range of
// column tiles (neighbouring tiles share cache lines of D).
#include "ircur_device.h"

namespace ircur {

namespace {

template <typename F> struct Mma;
template <> struct Mma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // row of the 16 x 16 accumulator held by lane l in register v (column l % 16)
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <> struct Mma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};

// Row tiles whose D entries a wave requests together: 6 with 32-bit
// arithmetic, 4 in FP64 (twice the registers per value); the wide variant
// takes 9, so that with up to 288 sampled rows (18 tiles, 9 per wave) every
// wave makes a single round trip to memory.
template <typename F> struct GroupTiles { static constexpr int value = 6; };
template <> struct GroupTiles<double> { static constexpr int value = 4; };
constexpr int kWideTiles = 9;

}  // namespace

size_t pass16_lds_bytes(int dtype, int R, int s) {
    (void)dtype;
    (void)R;
    const size_t red = 2 * 4 * 64 * sizeof(double) + (2 * 2 * 64 + 2) * sizeof(double);
    const size_t idx = ((size_t)s + 15) / 16 * 16 * sizeof(int32_t);
    return idx > red ? idx : red;
}

bool pass16_ok(int dtype, int R, int smax) {
    (void)dtype;
    return R >= kPass16MinRank && R <= kPass16MaxRank && smax <= kPass16MaxRows;
}

namespace {

template <typename T, typename F, int R, bool LIT, int GT>
__device__ __forceinline__ void pass16_side(const SideArgs& S, int tile, double zeta, float zeta_f, char* lds) {
    typedef Mma<F> M;
    typedef typename M::v4 v4;
    constexpr int KR = (R + 3) / 4;                  // k-steps over the factor index
    constexpr int NB = (2 * KR + 4) * 64;            // operand block of one row tile
    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ct = w & 1, rh = w >> 1;               // column tile of the wave, half of the row tiles
    const int64_t n = S.n;
    const int64_t j = (int64_t)tile * 32 + ct * 16 + (l & 15);
    const bool jv = j < n;
    const int64_t jc = jv ? j : n - 1;               // loads stay in bounds; the values are masked
    const T* __restrict__ X = (const T*)S.X;
    const F* __restrict__ P = (const F*)S.P;
    const F* __restrict__ tb = (const F*)S.tiled;
    const int32_t* __restrict__ rows = S.rows;
    const int64_t ldX = S.ldX;
    const int s = S.s;
    const int nrt = (s + 15) >> 4;
    int32_t* srows = (int32_t*)lds;                  // nrt * 16 sampled row indices

    // the sampled row indices in LDS (padded to whole tiles with the first one)
    for (int e = tid; e < nrt * 16; e += 256) srows[e] = rows[e < s ? e : 0];
    // B operand of the products with the factor: P[4 ks + l / 16][j]
    F pB[KR];
#pragma unroll
    for (int ks = 0; ks < KR; ++ks) {
        const int c = 4 * ks + (l >> 4);
        const F v = P[(c < R ? c : 0) * n + jc];
        pB[ks] = (c < R && jv) ? v : F(0);
    }
    // operands of the output map (used by the first row half's waves)
    F gA[KR], tA[4];
    {
        const F* __restrict__ Gm = (const F*)S.Gm;
        const F* __restrict__ Tm = (const F*)S.outmat;
        const int m = l & 15;
#pragma unroll
        for (int ks = 0; ks < KR; ++ks) {
            const int c = 4 * ks + (l >> 4);
            const F g = Gm[(m < R ? m : 0) * R + (c < R ? c : 0)];
            gA[ks] = (m < R && c < R) ? g : F(0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int dr = M::row(l, v);
            const F t = Tm ? Tm[(dr < R ? dr : 0) * R + (m < R ? m : 0)] : F(0);
            tA[v] = (dr < R && m < R) ? t : F(0);
        }
    }
    __syncthreads();
    // two accumulators (tiles of even and odd position in a group), added at the end
    v4 acc0 = {F(0), F(0), F(0), F(0)}, acc1 = acc0;
    F zz = F(0), dd = F(0);
    // the wave's row tiles rh, rh + 2, ..., GT at a time: the D entries and the
    // operand blocks of a group are requested together (the blocks are laid
    // out in lane order by the SVD, so each is one coalesced load per k-step)
    for (int g0 = rh; g0 < nrt; g0 += 2 * GT) {
        F d[GT][4], q1[GT][KR], q3[GT][KR], q2[GT][4];
#pragma unroll
        for (int u = 0; u < GT; ++u) {
            const int rt = g0 + 2 * u;
            const int rr = rt < nrt ? rt : rh;       // (a valid tile; masked below)
            const int a0 = rr * 16;
#pragma unroll
            for (int v = 0; v < 4; ++v) d[u][v] = ld<T, F>(X + (int64_t)srows[a0 + M::row(l, v)] * ldX + jc);
            const F* bk = tb + (size_t)rr * NB + l;
#pragma unroll
            for (int ks = 0; ks < KR; ++ks) {
                q1[u][ks] = bk[ks * 64];
                if (LIT) q3[u][ks] = bk[(KR + ks) * 64];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) q2[u][v] = bk[(2 * KR + v) * 64];
        }
#pragma unroll
        for (int u = 0; u < GT; ++u) {
            const int rt = g0 + 2 * u;
            if (rt >= nrt) continue;                 // uniform
            const int a0 = rt * 16;
            v4 dot = {F(0), F(0), F(0), F(0)};
#pragma unroll
            for (int ks = 0; ks < KR; ++ks) dot = M::mma(q1[u][ks], pB[ks], dot);
            v4 xr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const F dv = (a0 + M::row(l, v) < s && jv) ? d[u][v] : F(0);
                const F x = dv - dot[v];
                xr[v] = above(x < F(0) ? -x : x, zeta, zeta_f) ? F(0) : x;
                dd = fmaT(dv, dv, dd);
            }
            if (u & 1) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc1 = M::mma(q2[u][v], xr[v], acc1);
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc0 = M::mma(q2[u][v], xr[v], acc0);
            }
            if (LIT) {
                v4 z = xr;
#pragma unroll
                for (int ks = 0; ks < KR; ++ks) z = M::mma(q3[u][ks], pB[ks], z);
#pragma unroll
                for (int v = 0; v < 4; ++v) zz = fmaT(z[v], z[v], zz);
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) zz = fmaT(xr[v], xr[v], zz);
            }
        }
    }
    v4 acc = acc0 + acc1;

    // the two row halves of each column tile meet in LDS; the first half's
    // wave adds and writes its 16 columns
    __syncthreads();
    F* sacc = (F*)lds;                               // 2 x 4 x 64
    double* szd = (double*)(lds + 2 * 4 * 64 * sizeof(double));   // 2 x 2 x 64, then 2 results
    if (rh == 1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) sacc[(ct * 4 + v) * 64 + l] = acc[v];
        szd[(ct * 2) * 64 + l] = (double)zz;
        szd[(ct * 2 + 1) * 64 + l] = (double)dd;
    }
    __syncthreads();
    double res = 0.0, dsum = 0.0;
    if (rh == 0) {
        double zl = (double)zz, dl = (double)dd;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += sacc[(ct * 4 + v) * 64 + l];
        zl += szd[(ct * 2) * 64 + l];
        dl += szd[(ct * 2 + 1) * 64 + l];
        // val = Gm P + acc; out = Tm^T val (the k-steps of the second product
        // are the accumulator rows of val, as above)
        v4 val = acc;
#pragma unroll
        for (int ks = 0; ks < KR; ++ks) val = M::mma(gA[ks], pB[ks], val);
        v4 o = val;
        if (S.outmat) {
            o = v4{F(0), F(0), F(0), F(0)};
#pragma unroll
            for (int v = 0; v < 4; ++v) o = M::mma(tA[v], val[v], o);
        }
        F* __restrict__ out = (F*)S.out;
        double corr = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = M::row(l, v);
            if (c < R && jv) {
                out[c * n + j] = o[v];
                if (LIT) corr = __builtin_fma((double)acc[v], (double)acc[v], corr);
            }
        }
        res = wave_sum(zl - corr);
        dsum = wave_sum(dl);
    }
    __syncthreads();
    if (rh == 0 && ct == 1 && l == 0) {
        szd[256] = res;
        szd[257] = dsum;
    }
    __syncthreads();
    if (w == 0 && l == 0) {
        S.part[2 * tile] = res + szd[256];
        S.part[2 * tile + 1] = dsum + szd[257];
    }
}

template <typename T, typename F, int R, bool LIT, int GT>
__device__ __forceinline__ void pass16_body(const PassArgs& a, char* lds) {
    if (a.st->stop) return;
    // XCD-aware order: workgroups are dealt to the 8 XCDs in turn, so item
    // b = xcd * per + slot gives each XCD a contiguous range of column tiles
    const int nt0 = a.side[0].nwg;
    const int nt = nt0 + a.side[1].nwg;
    const int per = (int)(gridDim.x >> 3);
    const int b = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (b >= nt) {
        if (b == nt && a.gapT) gap_estimate(a.gapT, a.gapinfo, a.gapR, (double*)lds);   // (a spare workgroup)
        return;
    }
    if (b < nt0) pass16_side<T, F, R, LIT, GT>(a.side[0], b, a.zeta, a.zeta_f, lds);
    else pass16_side<T, F, R, LIT, GT>(a.side[1], b - nt0, a.zeta, a.zeta_f, lds);
}

template <typename T, typename F, int R, bool LIT>
__global__ __launch_bounds__(256) void pass16_kernel(PassArgs a) {
    extern __shared__ char lds[];
    pass16_body<T, F, R, LIT, GroupTiles<F>::value>(a, lds);
}

// The wide variant (32-bit arithmetic, padded rank at most 12, at most 288
// sampled rows per side): every wave's loads in one group, with the register
// budget of three waves per SIMD (as many as the launch needs at n = 10^4;
// padded rank 16 would need more).
template <typename T, typename F, int R, bool LIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 3))) void pass16_wide_kernel(PassArgs a) {
    extern __shared__ char lds[];
    pass16_body<T, F, R, LIT, kWideTiles>(a, lds);
}

template <typename T, typename F, int R>
hipError_t pass16_r(const PassArgs& a, hipStream_t s) {
    const unsigned nb = (unsigned)(a.side[0].nwg + a.side[1].nwg) + (a.gapT ? 1 : 0);
    const unsigned grid = (nb + 7) / 8 * 8;          // a whole number of rounds over the 8 XCDs
    const int smax = std::max(a.side[0].s, a.side[1].s);
    const size_t lds = pass16_lds_bytes(0, R, smax);
    if constexpr (sizeof(F) == 4 && R <= 12) {
        if ((smax + 15) / 16 <= 2 * kWideTiles) {
            if (a.err_mode == 0) pass16_wide_kernel<T, F, R, true><<<grid, 256, lds, s>>>(a);
            else pass16_wide_kernel<T, F, R, false><<<grid, 256, lds, s>>>(a);
            return hipGetLastError();
        }
    }
    if (a.err_mode == 0) pass16_kernel<T, F, R, true><<<grid, 256, lds, s>>>(a);
    else pass16_kernel<T, F, R, false><<<grid, 256, lds, s>>>(a);
    return hipGetLastError();
}

// (padded ranks 8..16 only: smaller ranks take the vector pass)
#define IRCUR_RANK_SWITCH16(FN, T, F, R, ...)                   \
    switch (R) {                                                \
        case 8: return FN<T, F, 8>(__VA_ARGS__);                \
        case 10: return FN<T, F, 10>(__VA_ARGS__);              \
        case 12: return FN<T, F, 12>(__VA_ARGS__);              \
        case 16: return FN<T, F, 16>(__VA_ARGS__);              \
        default: return hipErrorInvalidValue;                   \
    }

}  // namespace

hipError_t launch_pass16(const PassArgs& a, int dtype, int R, hipStream_t s) {
    if (dtype == 0) { IRCUR_RANK_SWITCH16(pass16_r, double, double, R, a, s) }
    if (dtype == 1) { IRCUR_RANK_SWITCH16(pass16_r, float, float, R, a, s) }
    if (dtype == 2) { IRCUR_RANK_SWITCH16(pass16_r, bf16_t, float, R, a, s) }
    return hipErrorInvalidValue;
}

}  // namespace ircur
