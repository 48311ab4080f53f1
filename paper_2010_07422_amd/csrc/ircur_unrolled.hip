// Unrolled, differentiable IRCUR over a batch of independent instances.
//
// The paper's iteration (Algorithm 1) uses the hard threshold of eq. (4).
// The unrolled mode runs K iterations with one threshold zeta_k per
// iteration and the gate S(x) = x g, g = sigmoid((|x| - zeta) / (tau_rel zeta))
// (tau_rel = 0: eq. (4) exactly), so that a loss of the final estimate is
// differentiable in the zeta_k.  Per instance,
//     loss = ||A_K B_K - W* V*^T||_F / ||W* V*^T||_F .
//
// Forward, per step k (one launch per stage for the whole batch):
//   ucore   M = [D - S]_{I,J} with the gated S (and the two MFMA layouts)
//   svd     the batched Phase II core kernel (factored pseudo-inverse)
//   upass   A_{k+1} = C Q Ly^-T, B_{k+1} = Wt^T R with the same gate
// then the loss from factor Grams.
//
// Reverse, per step k = K-1 .. 0, from Abar = dloss/dA_{k+1}, Bbar = dloss/dB_{k+1}:
//   ubpass(1)  Wbar = R Bbar^T (sI x R) and Tbar = C^T Abar (sJ x R), recomputing
//              the gathered rows and columns of this step from D
//   ubsmall    adjoint of the core, two workgroups per instance (the W-side and
//              the V-side solves run concurrently): singular triplets
//              of H_r(M) from Kc, the projections P1 = V_r^T Ubar = Sigma U_k^T Wbar^T
//              and P2 = Ubar W_r = Tbar U_k of the adjoint of U^+, resolvent solves
//              (sigma_c^2 I - M_perp M_perp^T) x = P1 (and the M^T M side) by
//              conjugate gradients on the complement of the top-r subspaces, and
//              Mbar = X1 V_r^T + W_r X2^T (first-order perturbation of the
//              truncated pseudo-inverse)
//   ubpass(2)  the gate adjoint: dloss/dzeta_k, Abar_k and Bbar_k
//   ubreduce   adds the per-row partials of Abar_k[I, :], Bbar_k[:, J] and zeta.
#include "ircur_device.h"
#include "ircur_small.h"

#include <stdint.h>
#include <type_traits>

namespace ircur {

namespace {

__device__ __forceinline__ int find_inst(const int32_t* __restrict__ off, int nb, int x) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ float round_down_f(double z) {
    float f = (float)z;
    if ((double)f > z) f = nextafterf(f, -__builtin_inff());
    return f;
}

// S = x g and its derivatives: g, dS/dx, dS/dzeta, with tauz = tau_rel zeta
// passed as the launch-uniform reciprocals itz = 1 / tauz and
// itzz = 1 / (tauz zeta), so that an entry costs one division (that of g).
template <typename F>
__device__ __forceinline__ void gate_derivs(F x, F zeta, F itz, F itzz, F& g, F& dSdx, F& dSdz) {
    const F ax = x < F(0) ? -x : x;
    g = F(1) / (F(1) + exp_t((zeta - ax) * itz));
    const F gg = g * (F(1) - g);
    dSdx = g + ax * gg * itz;
    dSdz = -x * ax * gg * itzz;
}

// ------------------------------------------------------------ forward ---

template <typename T, typename F, int R, bool GATE>
__global__ __launch_bounds__(256) void ucore_kernel(const CoreArgs* __restrict__ arr, const int32_t* __restrict__ off,
                                                    int nb, const double* __restrict__ zk, double tau_rel) {
    const int b = find_inst(off, nb, blockIdx.x);
    const CoreArgs& a = arr[b];
    const int local = blockIdx.x - off[b];
    if (local == 0 && threadIdx.x == 0) a.st->bar_ctr = 0u;
    const int64_t idx = (int64_t)local * 256 + threadIdx.x;
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
    const double zeta = *zk;
    F v;
    if (GATE) {
        const F x = d - dot;
        v = d - x * gate_value<F>(x, (F)zeta, (F)(tau_rel * zeta));
    } else {
        bool o;
        v = entry_value<F>(d, dot, zeta, round_down_f(zeta), &o);
    }
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

template <typename T, typename F, int R, bool GATE>
__global__ __launch_bounds__((64 * PassWaves<T, R>::value)) void upass_kernel(const PassArgs* __restrict__ arr,
                                                               const int32_t* __restrict__ off, int nb,
                                                               const double* __restrict__ zk, double tau_rel) {
    __shared__ F red[PassTree<T, F, R>::nred];
    __shared__ double redzd[PassTree<T, F, R>::nzd];
    const int b = find_inst(off, nb, blockIdx.x);
    const PassArgs& a = arr[b];
    const int local = blockIdx.x - off[b];
    const double zeta = *zk;
    const float zf = round_down_f(zeta);
    const F tz = (F)(tau_rel * zeta);
    if (local < a.side[0].nwg)
        side_body<T, F, R, false, GATE>(a.side[0], local, 0, zeta, zf, red, redzd, tz);
    else
        side_body<T, F, R, false, GATE>(a.side[1], local - a.side[0].nwg, 0, zeta, zf, red, redzd, tz);
}

// ---------------------------------------------------------------- loss ---

constexpr int kGramRows = 128;

template <typename F>
__global__ __launch_bounds__(256) void ugram_kernel(const ULoss* __restrict__ arr, const int32_t* __restrict__ off,
                                                    int nb) {
    __shared__ double ys[kGramRows][33];
    const int b = find_inst(off, nb, blockIdx.x);
    const ULoss& L = arr[b];
    const int local = blockIdx.x - off[b];
    const int side = local < L.nwgA ? 0 : 1;
    const int w = side == 0 ? local : local - L.nwgA;
    const int nw = side == 0 ? L.nwgA : L.nwgB;
    const int64_t n = side == 0 ? L.n1 : L.n2;
    const F* __restrict__ X = (const F*)(side == 0 ? L.At : L.B);   // R x n
    const F* __restrict__ S = (const F*)(side == 0 ? L.Ws : L.Vs);  // n x r
    const int R = L.R, r = L.r, R2 = 2 * R;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t ch = w; ch * kGramRows < n; ch += nw) {
        const int t = threadIdx.x;
        if (t < kGramRows) {
            const int64_t i = ch * kGramRows + t;
            for (int c = 0; c < R; ++c) {
                ys[t][c] = i < n ? (double)X[c * n + i] : 0.0;
                ys[t][R + c] = (i < n && c < r) ? (double)S[i * r + c] : 0.0;
            }
        }
        __syncthreads();
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q;
            if (e < R2 * R2) {
                const int c = e / R2, d = e - c * R2;
                double s = acc[q];
                for (int row = 0; row < kGramRows; ++row) s = __builtin_fma(ys[row][c], ys[row][d], s);
                acc[q] = s;
            }
        }
        __syncthreads();
    }
    double* out = L.gpart + (size_t)local * R2 * R2;
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e < R2 * R2) out[e] = acc[q];
    }
}

// One workgroup per instance: reduce the Gram partials; the loss from
//   ||A B||^2 = <A^T A, B B^T>,  <A B, W* V*^T> = <A^T W*, B V*>,
//   ||W* V*^T||^2 = <W*^T W*, V*^T V*>.
__global__ __launch_bounds__(256) void uloss_kernel(const ULoss* __restrict__ arr) {
    __shared__ double part[3][256];
    const ULoss& L = arr[blockIdx.x];
    const int R = L.R, r = L.r, R2 = 2 * R, Q2 = R2 * R2;
    for (int e = threadIdx.x; e < 2 * Q2; e += 256) {
        const int side = e / Q2, f = e - side * Q2;
        const int w0 = side == 0 ? 0 : L.nwgA, w1 = side == 0 ? L.nwgA : L.nwgA + L.nwgB;
        double s = 0.0;
        for (int w = w0; w < w1; ++w) s += L.gpart[(size_t)w * Q2 + f];
        L.gsum[e] = s;
    }
    __syncthreads();
    const double* GA = L.gsum;
    const double* GB = L.gsum + Q2;
    double ab = 0.0, cr = 0.0, ls = 0.0;
    for (int e = threadIdx.x; e < Q2; e += 256) {
        const int c = e / R2, d = e - c * R2;
        if (c < R && d < R) ab = __builtin_fma(GA[e], GB[e], ab);
        else if (c < R && d >= R && d - R < r) cr = __builtin_fma(GA[e], GB[e], cr);
        else if (c >= R && d >= R && c - R < r && d - R < r) ls = __builtin_fma(GA[e], GB[e], ls);
    }
    part[0][threadIdx.x] = ab;
    part[1][threadIdx.x] = cr;
    part[2][threadIdx.x] = ls;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < 3; ++q) part[q][threadIdx.x] += part[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double e2 = part[0][0] - 2.0 * part[1][0] + part[2][0];
        const double l2 = part[2][0];
        const double loss = l2 > 0.0 ? __builtin_sqrt((e2 > 0.0 ? e2 : 0.0) / l2) : 0.0;
        L.loss[0] = loss;
        L.gsum[2 * Q2] = loss;
        L.gsum[2 * Q2 + 1] = l2;
    }
}

// dloss/dA_K = s (A G_BB - W* (B V*)^T),  dloss/dB_K = s (G_AA B - (A^T W*) V*^T),
// s = dloss_b / (||E|| ||L*||).
template <typename F>
__global__ __launch_bounds__(256) void ulossadj_kernel(const ULoss* __restrict__ arr, const int32_t* __restrict__ off,
                                                       int nb, const double* __restrict__ dloss) {
    const int b = find_inst(off, nb, blockIdx.x);
    const ULoss& L = arr[b];
    const int local = blockIdx.x - off[b];
    const int R = L.R, r = L.r, R2 = 2 * R, Q2 = R2 * R2;
    const int nA = (int)((L.n1 + 255) / 256);
    const double loss = L.gsum[2 * Q2], l2 = L.gsum[2 * Q2 + 1];
    const double den = loss * l2;                       // ||E|| ||L*|| = loss ||L*||^2
    const double sc = (den > 0.0 ? 1.0 / den : 0.0) * (dloss ? dloss[b] : 1.0);
    const int side = local < nA ? 0 : 1;
    const int64_t n = side == 0 ? L.n1 : L.n2;
    const int64_t i = (int64_t)(side == 0 ? local : local - nA) * 256 + threadIdx.x;
    if (i >= n) return;
    const double* G = L.gsum + (side == 0 ? Q2 : 0);   // side A uses G_B, side B uses G_A
    const F* __restrict__ X = (const F*)(side == 0 ? L.At : L.B);
    const F* __restrict__ S = (const F*)(side == 0 ? L.Ws : L.Vs);
    F* __restrict__ out = (F*)(side == 0 ? L.Abar : L.Bbar);
    double x[32], sv[32];
    for (int c = 0; c < R; ++c) x[c] = (double)X[c * n + i];
    for (int f = 0; f < r; ++f) sv[f] = (double)S[i * r + f];
    for (int c = 0; c < R; ++c) {
        double v = 0.0;
        for (int e = 0; e < R; ++e) v = __builtin_fma(x[e], G[e * R2 + c], v);
        for (int f = 0; f < r; ++f) v = __builtin_fma(-sv[f], G[c * R2 + R + f], v);
        out[c * n + i] = (F)(sc * v);
    }
}

// ------------------------------------------------------------ reverse ---

// Phase 1: per sampled row a (column b) the partial sums over this block's
// 64 outputs of  R[a, j] Bbar[c, j]  (C[i, b] Abar[i, c]).
// Phase 2: the gate adjoint.  Row side, output j:
//     Rbar[a, j] = Wt[a, :] Bbar[:, j] + (j = J_b ? X1[a, :] V_r[b, :] + W_r[a, :] X2[b, :] : 0)
//     Xbar = -Rbar dS/dx,  zeta_bar += -Rbar dS/dzeta,
//     Bbar_k[:, j] = -sum_a A_k[I_a, :]^T Xbar (dense),  Abar_k[I_a, :] partial -sum_j Xbar B_k[:, j]^T
// and the column side with Cbar[i, b] = Abar[i, :] Tp[b, :] and the roles of
// the factors exchanged.
constexpr int pow2_ceil(int v) { return v <= 1 ? 1 : 2 * pow2_ceil((v + 1) / 2); }
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Sum over the 64 lanes of V values per lane at once (V a power of two, at most
// 64), by recursive halving: at level i a lane keeps one half of its values
// (the upper half if lane bit halv_bit(i) is set) and adds its partner's copy
// of that half, the partner differing in that bit and agreeing in the bits of
// the earlier levels.  The first four levels (the largest) pair lanes within
// a row of 16 by DPP moves on the vector ALU: row_mirror (l ^ 15),
// row_half_mirror (l ^ 7), quad_perm (l ^ 2, l ^ 1); the last two take
// l ^ 16 (swizzle inside 32 lanes) and l ^ 32 (permute through LDS).  The six
// partner masks span all lane bits, so each final sum covers every lane.
// After log2 V levels lane l holds the whole sum of value halving_index(l);
// plain butterfly steps with the remaining partners finish smaller V.
// Values whose index modulo RP is RL or more are zero padding: the levels
// that split on the higher index bits leave them alone.  V - 1 exchanges at
// most instead of 6 V; the summation tree is fixed.
constexpr int halv_bit(int i) { return i < 4 ? 3 - i : i; }

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float swz16_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F));
}
__device__ __forceinline__ double swz16_f(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)u, 0x401F);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(u >> 32), 0x401F);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <int CTRL> __device__ __forceinline__ double dpp_any(double v) { return dpp_d<CTRL>(v); }
template <int CTRL> __device__ __forceinline__ float dpp_any(float v) { return dpp_f<CTRL>(v); }

// the partner's copy of v at level LV
template <int LV, typename F>
__device__ __forceinline__ F halv_partner(F v) {
    if constexpr (LV == 0) return dpp_any<0x140>(v);          // row_mirror
    else if constexpr (LV == 1) return dpp_any<0x141>(v);     // row_half_mirror
    else if constexpr (LV == 2) return dpp_any<0x4E>(v);      // quad_perm [2,3,0,1]
    else if constexpr (LV == 3) return dpp_any<0xB1>(v);      // quad_perm [1,0,3,2]
    else if constexpr (LV == 4) return swz16_f(v);
    else return __shfl_xor(v, 32, 64);
}

template <int CNT, int LV, int V, int RP, int RL, typename F>
struct HalvingLevel {
    static __device__ __forceinline__ void run(F (&a)[V], int lane) {
        constexpr int h = CNT / 2;
        const bool hi = ((lane >> halv_bit(LV)) & 1) != 0;
#pragma unroll
        for (int j = 0; j < h; ++j) {
            if (h >= RP && (j % RP) >= RL) continue;       // padding: zero on both sides
            const F send = hi ? a[j] : a[j + h];
            const F keep = hi ? a[j + h] : a[j];
            a[j] = keep + halv_partner<LV>(send);
        }
        HalvingLevel<h, LV + 1, V, RP, RL, F>::run(a, lane);
    }
};
template <int LV, int V, int RP, int RL, typename F>
struct HalvingLevel<1, LV, V, RP, RL, F> {
    static __device__ __forceinline__ void run(F (&)[V], int) {}
};

template <int LV, typename F>
__device__ __forceinline__ F halving_tail(F v) {
    if constexpr (LV >= 6) return v;
    else return halving_tail<LV + 1>(v + halv_partner<LV>(v));
}

template <int V, int RP = 1, int RL = 1, typename F>
__device__ __forceinline__ F halving_sum(F (&a)[V], int lane) {
    static_assert(V >= 1 && V <= 64 && (V & (V - 1)) == 0, "V must be a power of two <= 64");
    HalvingLevel<V, 0, V, RP, RL, F>::run(a, lane);
    return halving_tail<ilog2(V)>(a[0]);
}

// the value whose sum lane l holds after halving_sum<V>, and whether l is the
// one lane that holds it (the lanes whose butterfly bits are all zero)
template <int V>
__device__ __forceinline__ int halving_index(int lane) {
    int v = 0;
#pragma unroll
    for (int i = 0; i < ilog2(V); ++i) v = (v << 1) | ((lane >> halv_bit(i)) & 1);
    return v;
}
template <int V>
__device__ __forceinline__ bool halving_writer(int lane) {
    int m = 0;
#pragma unroll
    for (int i = ilog2(V); i < 6; ++i) m |= 1 << halv_bit(i);
    return (lane & m) == 0;
}

template <typename T, typename F, int R, bool GATE, int PH>
__global__ __launch_bounds__(256) void ubpass_kernel(const UBack* __restrict__ arr, const int32_t* __restrict__ off,
                                                     int nb, const double* __restrict__ zk, double tau_rel) {
    __shared__ F red[4][R][64];
    __shared__ double zred[4];
    extern __shared__ __align__(16) unsigned char dyn[];
    const int b = find_inst(off, nb, blockIdx.x);
    // the table read through the constant space, so that the compiler takes
    // its pointers as global ones (plain loads, not flat ones, whose waits
    // would also hold up the LDS reads)
    typedef const __attribute__((address_space(4))) UBack CUBack;
    CUBack& u = ((CUBack*)arr)[b];
    const int local = blockIdx.x - off[b];
    const double zeta = *zk;
    const float zf = round_down_f(zeta);
    const F zF = (F)zeta;
    const F itz = (F)(1.0 / (tau_rel * zeta));
    const F itzz = (F)(1.0 / (tau_rel * zeta * zeta));
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool rowside = local < u.nwg_row;
    const int wg = rowside ? local : local - u.nwg_row;
    const int64_t n = rowside ? u.n2 : u.n1;
    const int s = rowside ? u.sI : u.sJ;
    const int64_t col = (int64_t)wg * 64 + lane;
    const bool valid = col < n;
    const int64_t cc = valid ? col : 0;
    const T* __restrict__ X = (const T*)(rowside ? u.D : u.Dt);
    const int64_t ldX = rowside ? u.ldD : u.ldDt;
    const int32_t* __restrict__ rows = rowside ? u.I : u.J;
    const F* __restrict__ At = (const F*)u.At;
    const F* __restrict__ Bk = (const F*)u.B;
    const F* __restrict__ P = rowside ? Bk : At;
    const F* __restrict__ Pb = (const F*)(rowside ? u.Bbar1 : u.Abar1);
    const F* __restrict__ Qf = rowside ? At : Bk;
    const int64_t nq = rowside ? u.n1 : u.n2;
    double* __restrict__ part = rowside ? u.partI : u.partJ;

    // per-row data in LDS: the row index, the factor row q (R values) and, in
    // phase 2, Wt, X1, W_r (row side) or Tp (column side) of that row
    const int nxv = PH == 2 ? (rowside ? 3 * R : R) : 0;
    const int stride = R + nxv;
    int* rix = (int*)dyn;                                         // s ints
    F* qs = (F*)(dyn + (((size_t)s * sizeof(int) + 15) & ~(size_t)15));
    for (int e = tid; e < s; e += 256) rix[e] = rows[e];
    __syncthreads();
    // (the stride is R, 2R or 4R: each case with its own constant divisor)
    auto fill = [&](auto kst) {
        constexpr int ST = decltype(kst)::value;
        const int tot = s * ST;
        for (int base = tid; base < tot; base += 256 * 8) {
            F v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = base + q * 256;
                F x = F(0);
                if (e < tot) {
                    const int a = e / ST, c = e - a * ST;
                    if (c < R) {
                        x = Qf[c * nq + rix[a]];
                    } else if (PH == 2) {
                        const int k = c - R, which = k / R, cr = k - which * R;
                        const double* srcd = rowside ? (which == 0 ? u.Wt : (which == 1 ? u.X1 : u.Wr)) : u.Tp;
                        const int64_t ix = (int64_t)a * R + cr;
                        x = (F)(rowside && which == 1 ? srcd[ix] + u.X1b[ix] : srcd[ix]);   // X1 = X1a + X1b
                    }
                }
                v[q] = x;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = base + q * 256;
                if (e < tot) qs[e] = v[q];
            }
        }
    };
    if (PH == 1) fill(std::integral_constant<int, R>{});
    else if (rowside) fill(std::integral_constant<int, 4 * R>{});
    else fill(std::integral_constant<int, 2 * R>{});
    __syncthreads();

    F p[R], pb[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        p[c] = P[c * n + cc];
        pb[c] = Pb[c * n + cc];
    }
    F vb[R], xb[R];
    bool inJ = false;
    if (PH == 2 && rowside) {
        const int bp = valid ? u.posJ[col] : -1;
        inJ = bp >= 0;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            vb[c] = inJ ? (F)u.Vr[(int64_t)bp * R + c] : F(0);
            xb[c] = inJ ? (F)(u.X2[(int64_t)bp * R + c] + u.X2b[(int64_t)bp * R + c]) : F(0);   // X2a + X2b
        }
    }
    F acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = F(0);
    double zacc = 0.0;
    const int chunk = (s + 3) >> 2;
    const int a_begin = wave * chunk;
    const int a_end = min(s, a_begin + chunk);
    constexpr int U = 8;
    F nx[U];
    if (a_end > a_begin) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) nx[uu] = ld<T, F>(X + (int64_t)rix[min(a_begin + uu, a_end - 1)] * ldX + cc);
    }
    for (int a0 = a_begin; a0 < a_end; a0 += U) {
        F dv[U];
#pragma unroll
        for (int uu = 0; uu < U; ++uu) dv[uu] = nx[uu];
        if (a0 + U < a_end) {
#pragma unroll
            for (int uu = 0; uu < U; ++uu) nx[uu] = ld<T, F>(X + (int64_t)rix[min(a0 + U + uu, a_end - 1)] * ldX + cc);
        }
        F wv[U];    // per row: the value whose products with the column factors are summed
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
            const int a = a0 + uu;
            wv[uu] = F(0);
            if (a < a_end) {
                const F* q = qs + (size_t)a * stride;
                const F d = valid ? dv[uu] : F(0);
                F dot = F(0);
#pragma unroll
                for (int c = 0; c < R; ++c) dot = fmaT(q[c], p[c], dot);
                const F x = d - dot;
                F g, dSdx, dSdz;
                if (GATE) {
                    gate_derivs<F>(x, zF, itz, itzz, g, dSdx, dSdz);
                } else {
                    g = above(x < F(0) ? -x : x, zeta, zf) ? F(1) : F(0);
                    dSdx = g;
                    dSdz = F(0);
                }
                if (PH == 1) {
                    const F v = GATE ? d - x * g : (g != F(0) ? d - x : d);
                    wv[uu] = valid ? v : F(0);
                } else {
                    F ybar = F(0);
                    if (rowside) {
#pragma unroll
                        for (int c = 0; c < R; ++c) ybar = fmaT(q[R + c], pb[c], ybar);
                        if (inJ) {
#pragma unroll
                            for (int c = 0; c < R; ++c) {
                                ybar = fmaT(q[2 * R + c], vb[c], ybar);
                                ybar = fmaT(q[3 * R + c], xb[c], ybar);
                            }
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < R; ++c) ybar = fmaT(pb[c], q[R + c], ybar);
                    }
                    const F xbar = -ybar * dSdx;
                    if (valid) zacc += -(double)ybar * (double)dSdz;
#pragma unroll
                    for (int c = 0; c < R; ++c) acc[c] = fmaT(q[c], xbar, acc[c]);
                    wv[uu] = valid ? xbar : F(0);
                }
            }
        }
        // part[row][c] = sum over the 64 columns of wv * m[c] (m = Bbar resp. P),
        // RG rows at a time by recursive halving
        constexpr int RP = pow2_ceil(R);
        constexpr int VMAX = sizeof(F) == 8 ? 32 : 64;
        constexpr int RG = U * RP <= VMAX ? U : VMAX / RP;
        constexpr int V = RG * RP;
#pragma unroll
        for (int g0 = 0; g0 < U; g0 += RG) {
            F hv[V];
#pragma unroll
            for (int i = 0; i < RG; ++i) {
#pragma unroll
                for (int c = 0; c < RP; ++c) {
                    if (c < R) hv[i * RP + c] = wv[g0 + i] * (PH == 1 ? pb[c] : p[c]);
                    else hv[i * RP + c] = F(0);
                }
            }
            const F sum = halving_sum<V, RP, R>(hv, lane);
            const int idx = halving_index<V>(lane);
            const int row = a0 + g0 + idx / RP, c = idx % RP;
            if (halving_writer<V>(lane) && c < R && row < a_end)
                part[((int64_t)wg * s + row) * R + c] = PH == 1 ? (double)sum : -(double)sum;
        }
    }
    if (PH == 2) {
#pragma unroll
        for (int c = 0; c < R; ++c) red[wave][c][lane] = acc[c];
        const double zw = wave_sum(zacc);
        if (lane == 0) zred[wave] = zw;
        __syncthreads();
        if (wave == 0) {
            F* __restrict__ out = (F*)(rowside ? u.Bbar0 : u.Abar0);
            if (valid) {
#pragma unroll
                for (int c = 0; c < R; ++c)
                    out[c * n + col] = -(((red[0][c][lane] + red[1][c][lane]) + red[2][c][lane]) + red[3][c][lane]);
            }
            if (lane == 0) u.partz[local] = ((zred[0] + zred[1]) + zred[2]) + zred[3];
        }
    }
}

// ---- adjoint of the core (two workgroups per instance, one per side) -----

// Column dot products of two m x 16 LDS blocks (row stride 16), fixed order.
__device__ void coldot16(const double* A, const double* B, int m, double* part, double* out) {
    const int c = threadIdx.x & 15, pp = threadIdx.x >> 4;
    double s = 0.0;
    for (int a = pp; a < m; a += 16) s = __builtin_fma(A[a * 16 + c], B[a * 16 + c], s);
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 16) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += part[q * 16 + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// One-sided Jacobi SVD of the leading r x r block of K (16 x 16, LDS) by the
// first wave, lane i owning row i of K and of Vm.  On return the columns of
// K are U Sigma and Vm holds V.
__device__ void jacobi16(double* K, double* Vm, int r) {
    const int i = threadIdx.x;
    if (i < 64) {
        if (i < 16)
            for (int c = 0; c < 16; ++c) Vm[i * 16 + c] = (i == c) ? 1.0 : 0.0;
        for (int sweep = 0; sweep < 60; ++sweep) {
            int rot = 0;
            for (int pp = 0; pp < r - 1; ++pp) {
                for (int qq = pp + 1; qq < r; ++qq) {
                    const double kp = i < r ? K[i * 16 + pp] : 0.0, kq = i < r ? K[i * 16 + qq] : 0.0;
                    // column dot products over the r <= 16 rows (lanes 0-15), from lane 0
                    const double al = readlane_d(row16_sum(kp * kp), 0), be = readlane_d(row16_sum(kq * kq), 0),
                                 ga = readlane_d(row16_sum(kp * kq), 0);
                    if (!(fabs(ga) > 1e-15 * __builtin_sqrt(al * be))) continue;
                    ++rot;
                    const double zt = (be - al) / (2.0 * ga);
                    const double t = (zt >= 0.0 ? 1.0 : -1.0) / (fabs(zt) + __builtin_sqrt(1.0 + zt * zt));
                    const double cs = 1.0 / __builtin_sqrt(1.0 + t * t), sn = cs * t;
                    if (i < r) {
                        K[i * 16 + pp] = cs * kp - sn * kq;
                        K[i * 16 + qq] = sn * kp + cs * kq;
                        const double vp = Vm[i * 16 + pp], vq = Vm[i * 16 + qq];
                        Vm[i * 16 + pp] = cs * vp - sn * vq;
                        Vm[i * 16 + qq] = sn * vp + cs * vq;
                    }
                }
            }
            if (rot == 0) break;
        }
    }
    __syncthreads();
}

// C (m16 x 16) = op(A) B with A in global memory (TA: A is K x m16, read
// transposed) and B (K x 16) in LDS.  Each wave takes every fourth 16-row tile
// and works on up to four of them at once, so that the global operands of
// 4 x 8 k-steps are in flight together; rows of C at or past rows_valid are
// written as zero.
template <bool TA>
__device__ void mm_rows_gA(const gdouble* __restrict__ A, int lda, const double* B, double* C, int m16, int K,
                           int rows_valid) {
    constexpr int MT = 4;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int ntile = m16 >> 4;
    const int ii = l & 15, kk = l >> 4;
    for (int t0 = w; t0 < ntile; t0 += 4 * MT) {
        d4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
        for (int kb = 0; kb < K; kb += 32) {
            double av[MT][8], bv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = kb + 4 * u;
                bv[u] = k < K ? B[(k + kk) * 16 + ii] : 0.0;
            }
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int t = t0 + 4 * m;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = kb + 4 * u;
                    const int i = t * 16 + ii;
                    av[m][u] = (t < ntile && k < K) ? (TA ? A[(size_t)(k + kk) * lda + i] : A[(size_t)i * lda + k + kk])
                                                    : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (kb + 4 * u < K) {
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        if (t0 + 4 * m < ntile) acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m][u], bv[u], acc[m], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
            if (t0 + 4 * m < ntile) tile_store(C, 16, (t0 + 4 * m) * 16, 0, acc[m], rows_valid);
    }
}

// Conjugate gradients, one system per column c < r:
//     (sig2[c] I - A B) x_c = rhs_c    (op = A B: the two products of M_perp)
// on m16 x 16 LDS blocks X (solution), Rr (rhs in, residual out), Pp, AP,
// with Tm (mo16 x 16) for the inner product.  Returns 1 if some column did
// not reach the tolerance.
template <bool LEFT>
__device__ int cg_solve(const gdouble* Mp, int sI16, int sJ16, int sI, int sJ, const double* sig2, int r,
                        double* X, double* Rr, double* Pp, double* AP, double* Tm, double* part, double* cols,
                        int max_it, double tol) {
    const int m16 = LEFT ? sI16 : sJ16, m = LEFT ? sI : sJ;
    double* rr = cols;          // 16
    double* bb = cols + 16;
    double* pap = cols + 32;
    double* rn = cols + 48;
    double* flag = cols + 64;
    for (int e = threadIdx.x; e < m16 * 16; e += NT) {
        X[e] = 0.0;
        Pp[e] = Rr[e];
    }
    __syncthreads();
    coldot16(Rr, Rr, m16, part, rr);
    if (threadIdx.x < 16) bb[threadIdx.x] = rr[threadIdx.x];
    __syncthreads();
    int it = 0;
    int fail = 0;
    for (; it < max_it; ++it) {
        // convergence test (every thread reads the same LDS values)
        bool done = true;
        for (int c = 0; c < r; ++c)
            if (rr[c] > tol * tol * bb[c]) done = false;
        if (done) break;
        // AP = sig2 P - Mp (Mp^T P)   (LEFT)   or   sig2 P - Mp^T (Mp P)
        if (LEFT) {
            mm_rows_gA<true>(Mp, sJ16, Pp, Tm, sJ16, sI16, sJ);
            __syncthreads();
            mm_rows_gA<false>(Mp, sJ16, Tm, AP, sI16, sJ16, sI);
        } else {
            mm_rows_gA<false>(Mp, sJ16, Pp, Tm, sI16, sJ16, sI);
            __syncthreads();
            mm_rows_gA<true>(Mp, sJ16, Tm, AP, sJ16, sI16, sJ);
        }
        __syncthreads();
        // The operator's result sig2 P - AP is formed where it is used, and
        // each column sum is accumulated in the loop that produces its terms:
        // thread t owns the entries e = t (mod 256), rows t >> 4 (mod 16) of
        // column t & 15, so its partial sums run over the same entries in the
        // same order as coldot16's.
        const int cq = threadIdx.x & 15;
        const double sg = sig2[cq];
        const bool cl = cq < r;
        // pap = sum over the rows of P (sig2 P - AP)
        {
            double sp = 0.0;
            for (int e = threadIdx.x; e < m16 * 16; e += NT) {
                const double ap = (cl && (e >> 4) < m) ? __builtin_fma(sg, Pp[e], -AP[e]) : 0.0;
                sp = __builtin_fma(Pp[e], ap, sp);
            }
            part[threadIdx.x] = sp;
            __syncthreads();
            if (threadIdx.x < 16) {
                double t = 0.0;
                for (int q = 0; q < 16; ++q) t += part[q * 16 + threadIdx.x];
                pap[threadIdx.x] = t;
            }
            __syncthreads();
        }
        // X += al P, R -= al (sig2 P - AP), rn = column sums of R^2
        {
            const double al = (cl && pap[cq] > 0.0) ? rr[cq] / pap[cq] : 0.0;
            double sr = 0.0;
            for (int e = threadIdx.x; e < m16 * 16; e += NT) {
                const double ap = (cl && (e >> 4) < m) ? __builtin_fma(sg, Pp[e], -AP[e]) : 0.0;
                X[e] = __builtin_fma(al, Pp[e], X[e]);
                const double rv = __builtin_fma(-al, ap, Rr[e]);
                Rr[e] = rv;
                sr = __builtin_fma(rv, rv, sr);
            }
            part[threadIdx.x] = sr;
            __syncthreads();
            if (threadIdx.x < 16) {
                double t = 0.0;
                for (int q = 0; q < 16; ++q) t += part[q * 16 + threadIdx.x];
                rn[threadIdx.x] = t;
            }
            __syncthreads();
        }
        {
            const double be = (cl && rr[cq] > 0.0) ? rn[cq] / rr[cq] : 0.0;
            for (int e = threadIdx.x; e < m16 * 16; e += NT) Pp[e] = __builtin_fma(be, Pp[e], Rr[e]);
        }
        __syncthreads();
        // the new residual norms become the current ones (the two buffers
        // swap roles; every read of the old ones is behind the barrier above)
        double* const t = rr;
        rr = rn;
        rn = t;
    }
    if (it >= max_it) fail = 1;
    (void)flag;
    return fail;
}

#ifdef IRCUR_PHASE_PROFILE
#define UPHASE(i)                                                              \
    do {                                                                       \
        if (blockIdx.x == 0 && threadIdx.x == 0) {                             \
            const uint64_t t_ = __builtin_amdgcn_s_memrealtime();              \
            u.st->phase[i] += t_ - t_prev;                                     \
            t_prev = t_;                                                       \
        }                                                                      \
    } while (0)
#else
#define UPHASE(i) do { } while (0)
#endif

// Two workgroups per instance: both form the shared set-up (identical
// arithmetic, identical global writes), then workgroup 0 solves the W-side
// systems and workgroup 1 the V-side ones, each writing its own part of
// X1 = X1a + X1b and X2 = X2a + X2b (the consumer adds the two parts).
__global__ __launch_bounds__(256) void ubsmall_kernel(const UBack* __restrict__ arr, int max_it, double tol) {
    extern __shared__ double smem[];
    const UBack& u = arr[blockIdx.x >> 1];
    const int side = blockIdx.x & 1;
#ifdef IRCUR_PHASE_PROFILE
    uint64_t t_prev = __builtin_amdgcn_s_memrealtime();
#endif
    const int R = u.R, r = u.r, sI = u.sI, sJ = u.sJ;
    const int sI16 = ((sI + 15) / 16) * 16, sJ16 = ((sJ + 15) / 16) * 16;
    const int m16 = sI16 > sJ16 ? sI16 : sJ16;
    double* B0 = smem;                  // m16 x 16 each
    double* B1 = B0 + m16 * 16;
    double* B2 = B1 + m16 * 16;
    double* B3 = B2 + m16 * 16;
    double* B4 = B3 + m16 * 16;
    double* K = B4 + m16 * 16;          // 16 x 16
    double* Vm = K + 256;
    double* Uk = Vm + 256;
    double* Vk = Uk + 256;
    double* Urr = Vk + 256;
    double* part = Urr + 256;           // 256
    double* cols = part + 256;          // 80
    double* sig = cols + 80;            // 16
    double* sig2 = sig + 16;            // 16
    int* order = (int*)(sig2 + 16);     // 16
    const int tid = threadIdx.x;

    // singular triplets of H_r(M) = Wt Kc Q^T:  Kc = U_k Sigma V_k^T
    for (int e = tid; e < 256; e += NT) {
        const int i = e >> 4, j = e & 15;
        K[e] = (i < R && j < R) ? gp(u.Kc)[i * R + j] : 0.0;
    }
    __syncthreads();
    jacobi16(K, Vm, r);
    if (tid < 16) {
        double s2 = 0.0;
        for (int i = 0; i < r; ++i) s2 = __builtin_fma(K[i * 16 + tid], K[i * 16 + tid], s2);
        part[tid] = tid < r ? __builtin_sqrt(s2) : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        for (int c = 0; c < 16; ++c) order[c] = c;
        for (int x = 0; x < r; ++x)
            for (int y = x + 1; y < r; ++y)
                if (part[order[y]] > part[order[x]]) { const int t = order[x]; order[x] = order[y]; order[y] = t; }
        for (int c = 0; c < 16; ++c) {
            sig[c] = c < r ? part[order[c]] : 0.0;
            sig2[c] = sig[c] * sig[c];
        }
        if (!(sig[r - 1] > 2.220446049250313e-16 * (double)(sI > sJ ? sI : sJ) * sig[0]))
            __hip_atomic_fetch_or(u.flags, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    for (int e = tid; e < 256; e += NT) {
        const int i = e >> 4, c = e & 15;
        const bool ok = c < r && sig[c] > 0.0;
        Uk[e] = ok ? K[i * 16 + order[c]] / sig[c] : 0.0;
        Vk[e] = ok ? Vm[i * 16 + order[c]] : 0.0;
    }
    __syncthreads();
    UPHASE(9);
    // W_r = Wt U_k,  V_r = Q V_k,  Tp = Q Ly^-T
    for (int e = tid; e < sI * R; e += NT) {
        const int a = e / R, c = e - a * R;
        double s = 0.0;
        for (int f = 0; f < R; ++f) s = __builtin_fma(gp(u.Wt)[a * R + f], Uk[f * 16 + c], s);
        gp(u.Wr)[e] = s;
    }
    for (int e = tid; e < sJ * R; e += NT) {
        const int b = e / R, c = e - b * R;
        double s = 0.0, t = 0.0;
        for (int f = 0; f < R; ++f) {
            s = __builtin_fma(gp(u.Q)[b * R + f], Vk[f * 16 + c], s);
            if (side == 1) t = __builtin_fma(gp(u.Q)[b * R + f], gp(u.TAd)[f * R + c], t);
        }
        gp(u.Vr)[e] = s;
        if (side == 1) gp(u.Tp)[e] = t;
    }
    // Wbar = sum of row partials (sI x R) into B0, Tbar (sJ x R) into B1: one
    // thread per entry (a, c < R), the partials of 16 workgroups loaded
    // together and added in workgroup order
    for (int e = tid; e < m16 * 16; e += NT) {
        B0[e] = 0.0;
        B1[e] = 0.0;
    }
    __syncthreads();
    // (the W side needs only Wbar, the V side only Tbar)
    for (int e = tid + (side == 0 ? 0 : sI * R); e < (side == 0 ? sI * R : (sI + sJ) * R); e += NT) {
        const bool row = e < sI * R;
        const int ee = row ? e : e - sI * R;
        const int a = ee / R, c = ee - a * R;
        const int nw = row ? u.nwg_row : u.nwg_col, sn = row ? sI : sJ;
        const gdouble* __restrict__ pp = gp(row ? u.partI : u.partJ);
        double acc = 0.0;
        for (int w0 = 0; w0 < nw; w0 += 16) {
            double v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = w0 + q < nw ? pp[((int64_t)(w0 + q) * sn + a) * R + c] : 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) acc += v[q];
        }
        (row ? B0 : B1)[a * 16 + c] = acc;
    }
    __syncthreads();
    // P1t = Wbar U_k Sigma (sI x r), P2 = Tbar U_k (sJ x r)
    for (int e = tid; e < m16 * 16; e += NT) {
        const int a = e >> 4, c = e & 15;
        double s0 = 0.0, s1 = 0.0;
        if (c < r) {
            for (int f = 0; f < R; ++f) {
                s0 = __builtin_fma(B0[a * 16 + f], Uk[f * 16 + c], s0);
                s1 = __builtin_fma(B1[a * 16 + f], Uk[f * 16 + c], s1);
            }
        }
        B2[e] = (a < sI) ? s0 * sig[c] : 0.0;
        B3[e] = (a < sJ) ? s1 : 0.0;
    }
    __syncthreads();
    UPHASE(10);
    // W_r and V_r into LDS (B0, B1 are free until the solves), 8 entries per
    // thread in flight
    for (int e0 = tid; e0 < m16 * 16; e0 += NT * 8) {
        double w[8], v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = e0 + q * NT;
            const int a = e >> 4, c = e & 15;
            w[q] = (e < m16 * 16 && a < sI && c < r) ? gp(u.Wr)[a * R + c] : 0.0;
            v[q] = (e < m16 * 16 && a < sJ && c < r) ? gp(u.Vr)[a * R + c] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = e0 + q * NT;
            if (e < m16 * 16) {
                B0[e] = w[q];
                B1[(e & 15) * m16 + (e >> 4)] = v[q];   // V_r^T: lanes along b read consecutive words
            }
        }
    }
    __syncthreads();
    // Urr = P1 W_r (r x r); W_r^T P1t and V_r^T P2 (r x r)
    {
        const int c = tid >> 4, e = tid & 15;
        double s = 0.0, s0 = 0.0, s1 = 0.0;
        if (c < r && e < r) {
            if (side == 0) {                    // (the W side's maps)
#pragma unroll 8
                for (int a = 0; a < sI; ++a) {
                    s = __builtin_fma(B2[a * 16 + c], B0[a * 16 + e], s);
                    s0 = __builtin_fma(B0[a * 16 + c], B2[a * 16 + e], s0);
                }
            } else {                            // (the V side's)
#pragma unroll 8
                for (int b = 0; b < sJ; ++b) s1 = __builtin_fma(B1[c * m16 + b], B3[b * 16 + e], s1);
            }
        }
        Urr[tid] = s;
        K[tid] = s0;    // W_r^T P1t  (r x r)
        Vm[tid] = s1;   // V_r^T P2
    }
    // M_perp = M - W_r Sigma V_r^T (padded, global): each wave takes rows a
    // (4 at a time, 12 entries of M per lane in flight), lanes run along b.  A
    // lane keeps the V_r rows of its three columns in registers and takes
    // -W_r[a, :] Sigma once per row; all 16 columns are summed (W_r, V_r and
    // sigma are zero at and past r, so the extra terms add exact zeros).
    {
        const int w4 = tid >> 6, l64 = tid & 63;
        double vb[3][16];
#pragma unroll
        for (int jb = 0; jb < 3; ++jb) {
            const int bc = l64 + 64 * jb;
#pragma unroll
            for (int c = 0; c < 16; ++c) vb[jb][c] = bc < sJ16 ? B1[c * m16 + bc] : 0.0;
        }
        for (int a0 = w4; a0 < sI16; a0 += 16) {
            double mv[4][3];
#pragma unroll
            for (int ia = 0; ia < 4; ++ia)
#pragma unroll
                for (int jb = 0; jb < 3; ++jb) {
                    const int ar = a0 + 4 * ia, bc = l64 + 64 * jb;
                    mv[ia][jb] = (ar < sI && bc < sJ) ? gp(u.M)[(int64_t)ar * sJ + bc] : 0.0;
                }
#pragma unroll
            for (int ia = 0; ia < 4; ++ia) {
                const int ar = a0 + 4 * ia;
                if (ar < sI16) {
                    double wr[16];
#pragma unroll
                    for (int c = 0; c < 16; ++c) wr[c] = -B0[ar * 16 + c] * sig[c];
#pragma unroll
                    for (int jb = 0; jb < 3; ++jb) {
                        const int bc = l64 + 64 * jb;
                        if (bc < sJ16) {
                            double v = 0.0;
                            if (ar < sI && bc < sJ) {
                                v = mv[ia][jb];
#pragma unroll
                                for (int c = 0; c < 16; ++c) v = __builtin_fma(wr[c], vb[jb][c], v);
                            }
                            gp(u.Mperp)[(int64_t)ar * sJ16 + bc] = v;
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    // right-hand sides projected on the complements: P1t - W_r (W_r^T P1t) into
    // B4 (W side), P2 - V_r (V_r^T P2) kept in global P2 (V side)
    for (int e = tid; e < m16 * 16; e += NT) {
        const int a = e >> 4, c = e & 15;
        double w = 0.0, v = 0.0;
        if (c < r) {
            w = B2[e];
            v = B3[e];
#pragma unroll
            for (int f = 0; f < 16; ++f) {      // K, Vm are zero at and past r
                if (side == 0 && a < sI) w = __builtin_fma(-B0[a * 16 + f], K[f * 16 + c], w);
                if (side == 1 && a < sJ) v = __builtin_fma(-B1[f * m16 + a], Vm[f * 16 + c], v);
            }
        }
        B4[e] = (a < sI) ? w : 0.0;
        if (side == 1 && a < sJ && c < R) gp(u.P2)[a * R + c] = (c < r) ? v : 0.0;
    }
    __syncthreads();
    UPHASE(12);
    int fail = 0;
    if (side == 0) {
        // W side:  (sig_c^2 I - M_perp M_perp^T) x_c = rhs_c  (rhs in B4; B1 serves as scratch)
        fail |= cg_solve<true>(gp(u.Mperp), sI16, sJ16, sI, sJ, sig2, r, B0, B4, B2, B3, B1, part, cols, max_it, tol);
        UPHASE(13);
        // Qm = x / sigma (into B0), then M_perp^T Qm (sJ x 16) into B4
        for (int e = tid; e < m16 * 16; e += NT) {
            const int c = e & 15;
            B0[e] = (c < r && sig[c] > 0.0) ? B0[e] / sig[c] : 0.0;
        }
        __syncthreads();
        mm_rows_gA<true>(gp(u.Mperp), sJ16, B0, B4, sJ16, sI16, sJ);
        __syncthreads();
        UPHASE(14);
        // X1a = Qm Sigma - W_r Sigma^-1 Urr Sigma^-1,  X2a = M_perp^T Qm
        for (int e = tid; e < sI * R; e += NT) {
            const int a = e / R, c = e - a * R;
            double v = 0.0;
            if (c < r) {
                v = B0[a * 16 + c] * sig[c];
                for (int f = 0; f < r; ++f) v = __builtin_fma(-gp(u.Wr)[a * R + f], Urr[f * 16 + c] / (sig[f] * sig[c]), v);
            }
            gp(u.X1)[e] = v;
        }
        for (int e = tid; e < sJ * R; e += NT) {
            const int b = e / R, c = e - b * R;
            gp(u.X2)[e] = B4[b * 16 + c];
        }
    } else {
        // V side:  (sig_c^2 I - M_perp^T M_perp) y_c = rhs_c  (rhs from P2)
        for (int e = tid; e < m16 * 16; e += NT) {
            const int a = e >> 4, c = e & 15;
            B1[e] = (a < sJ && c < R) ? gp(u.P2)[a * R + c] : 0.0;
        }
        __syncthreads();
        fail |= cg_solve<false>(gp(u.Mperp), sI16, sJ16, sI, sJ, sig2, r, B0, B1, B2, B3, B4, part, cols, max_it, tol);
        for (int e = tid; e < m16 * 16; e += NT) {
            const int c = e & 15;
            B0[e] = (c < r && sig[c] > 0.0) ? B0[e] / sig[c] : 0.0;   // Um
        }
        __syncthreads();
        mm_rows_gA<false>(gp(u.Mperp), sJ16, B0, B4, sI16, sJ16, sI);   // M_perp Um (sI x 16)
        __syncthreads();
        // X1b = M_perp Um,  X2b = Um Sigma
        for (int e = tid; e < sI * R; e += NT) {
            const int a = e / R, c = e - a * R;
            gp(u.X1b)[e] = c < r ? B4[a * 16 + c] : 0.0;
        }
        for (int e = tid; e < sJ * R; e += NT) {
            const int b = e / R, c = e - b * R;
            gp(u.X2b)[e] = c < r ? B0[b * 16 + c] * sig[c] : 0.0;
        }
    }
    UPHASE(15);
    if (tid == 0 && fail) __hip_atomic_fetch_or(u.flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of nw partials p[0], p[stride], ..., added in index order; the loads
// are issued 16 at a time so that they are in flight together.
__device__ __forceinline__ double sum_strided(const double* __restrict__ p, int64_t stride, int nw) {
    double s = 0.0;
    for (int w0 = 0; w0 < nw; w0 += 16) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = w0 + q < nw ? p[(int64_t)(w0 + q) * stride] : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (w0 + q < nw) s += v[q];
    }
    return s;
}

template <typename F>
__global__ __launch_bounds__(256) void ubreduce_kernel(const UBack* __restrict__ arr, const int32_t* __restrict__ off,
                                                       int nb) {
    __shared__ double red[256];
    const int b = find_inst(off, nb, blockIdx.x);
    const UBack& u = arr[b];
    const int local = blockIdx.x - off[b];
    const int R = u.R;
    const int nI = (u.sI * R + 255) / 256, nJ = (u.sJ * R + 255) / 256;
    if (local < nI) {
        const int e = local * 256 + threadIdx.x;
        if (e < u.sI * R) {
            const int a = e / R, c = e - a * R;
            const double s = sum_strided(u.partI + (int64_t)a * R + c, (int64_t)u.sI * R, u.nwg_row);
            F* A0 = (F*)u.Abar0;
            const int64_t idx = (int64_t)c * u.n1 + u.I[a];
            A0[idx] = (F)((double)A0[idx] + s);
        }
    } else if (local < nI + nJ) {
        const int e = (local - nI) * 256 + threadIdx.x;
        if (e < u.sJ * R) {
            const int bb = e / R, c = e - bb * R;
            const double s = sum_strided(u.partJ + (int64_t)bb * R + c, (int64_t)u.sJ * R, u.nwg_col);
            F* B0 = (F*)u.Bbar0;
            const int64_t idx = (int64_t)c * u.n2 + u.J[bb];
            B0[idx] = (F)((double)B0[idx] + s);
        }
    } else {
        double s = 0.0;
        for (int w = threadIdx.x; w < u.nwg_row + u.nwg_col; w += 256) s += u.partz[w];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h >= 1; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) u.dz[0] = red[0];
    }
}

__global__ __launch_bounds__(256) void udzeta_kernel(const double* __restrict__ dz_inst, int nb, int K,
                                                     double* __restrict__ dzeta) {
    for (int k = threadIdx.x; k < K; k += 256) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += dz_inst[(int64_t)k * nb + b];
        dzeta[k] = s;
    }
}

// ----------------------------------------------------------- launchers ---

template <typename T, typename F, int R>
hipError_t ucore_r(const CoreArgs* arr, const int32_t* off, int nb, int total, const double* zk, double tau,
                   hipStream_t s) {
    if (tau > 0.0) ucore_kernel<T, F, R, true><<<total, 256, 0, s>>>(arr, off, nb, zk, tau);
    else ucore_kernel<T, F, R, false><<<total, 256, 0, s>>>(arr, off, nb, zk, tau);
    return hipGetLastError();
}

template <typename T, typename F, int R>
hipError_t upass_r(const PassArgs* arr, const int32_t* off, int nb, int total, const double* zk, double tau,
                   hipStream_t s) {
    if (tau > 0.0) upass_kernel<T, F, R, true><<<total, 64 * PassWaves<T, R>::value, 0, s>>>(arr, off, nb, zk, tau);
    else upass_kernel<T, F, R, false><<<total, 64 * PassWaves<T, R>::value, 0, s>>>(arr, off, nb, zk, tau);
    return hipGetLastError();
}

template <typename T, typename F, int R>
hipError_t ubpass_r(int phase, const UBack* arr, const int32_t* off, int nb, int total, int max_s, const double* zk,
                    double tau, hipStream_t s) {
    const size_t lds = (((size_t)max_s * sizeof(int) + 15) & ~(size_t)15) + (size_t)max_s * 4 * R * sizeof(F);
    const size_t stat = sizeof(F) * 4 * R * 64 + 4 * sizeof(double);      // the reduction arrays
    if (lds + stat > 160 * 1024) return hipErrorInvalidValue;
    const void* fns[4] = {(const void*)ubpass_kernel<T, F, R, false, 1>, (const void*)ubpass_kernel<T, F, R, true, 1>,
                          (const void*)ubpass_kernel<T, F, R, false, 2>, (const void*)ubpass_kernel<T, F, R, true, 2>};
    static size_t granted[4] = {0, 0, 0, 0};
    const int fi = (phase == 1 ? 0 : 2) + (tau > 0.0 ? 1 : 0);
    if (lds > 64 * 1024 && lds > granted[fi]) {
        hipError_t e = hipFuncSetAttribute(fns[fi], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        granted[fi] = lds;
    }
    if (phase == 1) {
        if (tau > 0.0) ubpass_kernel<T, F, R, true, 1><<<total, 256, lds, s>>>(arr, off, nb, zk, tau);
        else ubpass_kernel<T, F, R, false, 1><<<total, 256, lds, s>>>(arr, off, nb, zk, tau);
    } else {
        if (tau > 0.0) ubpass_kernel<T, F, R, true, 2><<<total, 256, lds, s>>>(arr, off, nb, zk, tau);
        else ubpass_kernel<T, F, R, false, 2><<<total, 256, lds, s>>>(arr, off, nb, zk, tau);
    }
    return hipGetLastError();
}

#define IRCUR_URANK_SWITCH(FN, T, F, R, ...)                    \
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
        default: return hipErrorInvalidValue;                   \
    }

}  // namespace

hipError_t launch_ucore(const CoreArgs* arr, const int32_t* off, int nb, int total, const double* zk, double tau,
                        int dtype, int R, hipStream_t s) {
    if (dtype == 0) { IRCUR_URANK_SWITCH(ucore_r, double, double, R, arr, off, nb, total, zk, tau, s) }
    if (dtype == 1) { IRCUR_URANK_SWITCH(ucore_r, float, float, R, arr, off, nb, total, zk, tau, s) }
    return hipErrorInvalidValue;
}

hipError_t launch_upass(const PassArgs* arr, const int32_t* off, int nb, int total, const double* zk, double tau,
                        int dtype, int R, hipStream_t s) {
    if (dtype == 0) { IRCUR_URANK_SWITCH(upass_r, double, double, R, arr, off, nb, total, zk, tau, s) }
    if (dtype == 1) { IRCUR_URANK_SWITCH(upass_r, float, float, R, arr, off, nb, total, zk, tau, s) }
    return hipErrorInvalidValue;
}

hipError_t launch_uloss(const ULoss* arr, const int32_t* off, int nb, int total, int dtype, hipStream_t s) {
    if (dtype == 0) ugram_kernel<double><<<total, 256, 0, s>>>(arr, off, nb);
    else ugram_kernel<float><<<total, 256, 0, s>>>(arr, off, nb);
    uloss_kernel<<<nb, 256, 0, s>>>(arr);
    return hipGetLastError();
}

hipError_t launch_ulossadj(const ULoss* arr, const int32_t* off, int nb, int total, const double* dloss, int dtype,
                           hipStream_t s) {
    if (dtype == 0) ulossadj_kernel<double><<<total, 256, 0, s>>>(arr, off, nb, dloss);
    else ulossadj_kernel<float><<<total, 256, 0, s>>>(arr, off, nb, dloss);
    return hipGetLastError();
}

hipError_t launch_ubpass(int phase, const UBack* arr, const int32_t* off, int nb, int total, int max_s,
                         const double* zk, double tau, int dtype, int R, hipStream_t s) {
    if (dtype == 0) { IRCUR_URANK_SWITCH(ubpass_r, double, double, R, phase, arr, off, nb, total, max_s, zk, tau, s) }
    if (dtype == 1) { IRCUR_URANK_SWITCH(ubpass_r, float, float, R, phase, arr, off, nb, total, max_s, zk, tau, s) }
    return hipErrorInvalidValue;
}

size_t ubsmall_lds_bytes(int max_s16) {
    return ((size_t)5 * max_s16 * 16 + 5 * 256 + 256 + 80 + 32) * sizeof(double) + 16 * sizeof(int);
}

hipError_t launch_ubsmall(const UBack* arr, int nb, int max_s16, int cg_max_it, double cg_tol, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)ubsmall_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const size_t lds = ubsmall_lds_bytes(max_s16);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    ubsmall_kernel<<<2 * nb, 256, lds, s>>>(arr, cg_max_it, cg_tol);
    return hipGetLastError();
}

hipError_t launch_ubreduce(const UBack* arr, const int32_t* off, int nb, int total, int dtype, hipStream_t s) {
    if (dtype == 0) ubreduce_kernel<double><<<total, 256, 0, s>>>(arr, off, nb);
    else ubreduce_kernel<float><<<total, 256, 0, s>>>(arr, off, nb);
    return hipGetLastError();
}

hipError_t launch_udzeta(const double* dz_inst, int nb, int K, double* dzeta, hipStream_t s) {
    udzeta_kernel<<<1, 256, 0, s>>>(dz_inst, nb, K, dzeta);
    return hipGetLastError();
}

}  // namespace ircur
