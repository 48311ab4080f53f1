// Phase I on the sampled block and Phase II of Algorithm 1 in one launch
// (FP64 subspace arithmetic, ranks r <= 16):
//
//   core    M = [D - S_{k+1}]_{I,J}, S_{k+1} = T_zeta[D - L_k] on the block
//           (eq. (4), (5)), gathered by the core launch on every compute
//           unit and loaded into LDS here: workgroup g owns the 16 rows
//           I_{16g .. 16g+15} of M;
//   svd     an orthonormal basis Q (|J| x 16) whose first r columns span the
//           top-r right singular subspace of M (section 3.1), by subspace
//           iteration on A = M^T M accelerated with Chebyshev filters;
//   output  the per-row data and small maps of the fused pass, in the
//           basis-free form U^+ = Q_r (Y^T Y)^-1 Y^T, Y = M Q_r (see
//           ircur_svd.hip for the identities).
//
// Subspace iteration.  The block X has 16 columns; the first r are the
// wanted subspace (Cholesky QR keeps the span of the leading columns, so the
// others never perturb it) and the remaining ones, pushed towards the next
// singular directions by the same filters, give Rayleigh quotients below
// sigma_{r+1}^2 that set the filter interval and the gap estimate.  Work
// proceeds in sweeps:
//   test    with X = Q orthonormal: Z = A Q, Gy = Q^T A Q; converged when
//           ||Z_r - Q_r Gy_rr||_F <= tol ||Gy_rr||_F (first r columns);
//   filter  otherwise m applications of the scaled three-term Chebyshev
//           recurrence (Zhou and Saad 2007) for the interval [0, b], b the
//           largest Rayleigh quotient of the extra columns, normalised at the
//           largest quotient of the wanted ones, then Cholesky QR;
// the test application is also the first filter step.  With b = 0 (no
// extra columns, or before the columns have separated) a step is a scaled
// power step, i.e. plain subspace iteration.
//
// One application of A: each workgroup forms Y_blk = M_blk X (16 x 16) and
// its partial Z_g = M_blk^T Y_blk (|J| x 16) on the matrix cores, publishes
// the partial, and after a grid barrier reduces its slice of row tiles of Z
// (and, on a test, the small Grams) in a fixed order, forms its slice of the
// next X, publishes it, and after a second barrier reads the whole next X.
// Data exchanged between workgroups uses device-scope stores and loads, so
// the barriers need no cache-wide fence.  Every workgroup holds the reduced
// small matrices and takes identical decisions.
#include "ircur_block16.h"
#include "ircur_device.h"

#include <stdint.h>

namespace ircur {

namespace {

constexpr int P = 16;

template <typename T> struct FactorOf;
template <> struct FactorOf<double> { typedef double type; };
template <> struct FactorOf<float> { typedef float type; };
template <> struct FactorOf<bf16_t> { typedef float type; };

__device__ __forceinline__ void st_dev(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier over the G workgroups (all resident: G is at most the number
// of compute units and each workgroup takes one).  Every thread's stores have
// completed before its workgroup is counted; the spin is bounded (a flag is
// raised on time-out and the kernel runs on, so every wave reaches its end).
__device__ void grid_sync(uint32_t* ctr, uint32_t target, int32_t* fail) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > (1u << 22)) {
                __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
}

// Sum over the G partials of one 256-double block (block index `blk` of each
// partial, partials `pstride` doubles apart), thread t summing entry t in
// partial order; loads issued 32 at a time (one round trip for G <= 32).
__device__ __forceinline__ double sum_parts(const double* base, size_t pstride, int G) {
    double s = 0.0;
    for (int g0 = 0; g0 < G; g0 += 32) {
        double v[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = g0 + u < G ? ld_dev(base + (size_t)(g0 + u) * pstride) : 0.0;
#pragma unroll
        for (int u = 0; u < 32; ++u) s += v[u];
    }
    return s;
}

// Two such sums with their loads issued together (32 of each at a time).
__device__ __forceinline__ void sum_parts2(const double* b1, size_t s1, const double* b2, size_t s2, int G, double& r1,
                                           double& r2) {
    double x = 0.0, y = 0.0;
    for (int g0 = 0; g0 < G; g0 += 32) {
        double v[32], w[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            v[u] = g0 + u < G ? ld_dev(b1 + (size_t)(g0 + u) * s1) : 0.0;
            w[u] = g0 + u < G ? ld_dev(b2 + (size_t)(g0 + u) * s2) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            x += v[u];
            y += w[u];
        }
    }
    r1 = x;
    r2 = y;
}

// Pseudo-random entry i of the starting block in [-1, 1): the 32-bit
// finaliser of MurmurHash3 applied to the salt plus i times the golden-ratio
// constant.
__device__ __forceinline__ double rnd_x0(uint64_t salt, int i) {
    uint32_t h = (uint32_t)salt ^ (uint32_t)(salt >> 32) ^ ((uint32_t)i * 0x9E3779B9u);
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return (double)h * (2.0 / 4294967296.0) - 1.0;
}

}  // namespace

// Phase timers of profile builds: 100 MHz ticks accumulated in registers of
// the first thread and written once at the end of the launch.
#ifdef IRCUR_PHASE_PROFILE
#define CPHASE(i)                                                             \
    do {                                                                      \
        const uint64_t t_ = __builtin_amdgcn_s_memrealtime();                 \
        ph_[i] += t_ - t_prev;                                                \
        t_prev = t_;                                                          \
    } while (0)
#else
#define CPHASE(i) do { } while (0)
#endif

struct QTimes { uint64_t g, c, x; };

// M block in LDS: k-step ks (4 columns of M) holds its 4 x 16 entries with a
// column stride of 17 doubles, so that both the row-tiled reads of M X and
// the column-tiled reads of M^T Y fall on distinct banks.
__device__ __forceinline__ int mb_index(int row, int col) { return (col >> 2) * 68 + (col & 3) * 17 + row; }

namespace {

// Cholesky QR of the first `live` columns of X (rows >= rows_valid zero):
// X <- X L^-T with X^T X = L L^T.  A column is dead when its pivot falls to
// 1e-14 of its own squared norm (a column that is merely small after a power
// step is not mistaken for a dependent one).  A second pass runs when the
// first pivots of the wanted columns (the first nw), relative to the column
// norms, spread by more than `kappa2_one` (the rounding of X^T X would show
// in their orthogonality; the leading columns of the result depend only on
// the leading columns of X, and the extra columns' orthogonality only sets
// the filter interval) and whenever a column was found dependent (refilled
// with pseudo-random entries); at most four passes.  Gs, LiT: 16 x XS; st:
// 4; scr: 4 x 256.
__device__ __forceinline__ QTimes cholqr(double* X, int sJ16, int rows_valid, int live, int nw, double kappa2_one,
                                         int min_passes, double* Gs, double* LiT, int* dead, double* st, double* scr,
                                         uint64_t salt) {
    const int KS = sJ16 / 4, nt = sJ16 / 16;
    int need = min_passes;
    QTimes qt = {0, 0, 0};
#ifdef IRCUR_PHASE_PROFILE
    uint64_t t_ = __builtin_amdgcn_s_memrealtime();
#define QPHASE(f) do { const uint64_t n_ = __builtin_amdgcn_s_memrealtime(); qt.f += n_ - t_; t_ = n_; } while (0)
#else
#define QPHASE(f) do { } while (0)
#endif
    for (int pass = 0; pass < 4; ++pass) {
        gram16(X, KS, scr, Gs);
        QPHASE(g);
        chol16(Gs, XS, live, 1e-14, true, nullptr, LiT, dead, st, scr, nw);
        QPHASE(c);
        xmul16(X, nt, LiT);
        QPHASE(x);
        const int nd = (int)st[0];
        if (pass == 0 && st[2] > 0.0 && st[1] > kappa2_one * st[2]) need = max(need, 2);
        if (nd > 0) {
            need = max(need, pass + 2);
            for (int e = threadIdx.x; e < rows_valid * 16; e += NT) {
                const int b = e >> 4, c = e & 15;
                if (c < live && dead[c]) X[b * XS + c] = rnd_unit(salt ^ (0x5bd1e995ull * (uint64_t)(pass + 1)), (uint64_t)e);
            }
            __syncthreads();
        }
        if (pass + 1 >= need) break;
    }
    return qt;
}

}  // namespace

size_t csvd_lds_bytes(int sJ, int G) {
    const size_t sJ16 = ((size_t)sJ + 15) / 16 * 16;
    const size_t ntj = sJ16 / 16;
    const size_t tpg = (ntj + G - 1) / G;
    size_t d = 0;
    d += 17 * sJ16;                   // M block (padded operand order)
    d += sJ16 * XS;                   // X
    d += 3 * tpg * 256;               // X_{j-1} slice, reduced Z slice, B_k[:, J] of the slice
    d += 2 * 256;                     // Y, A_k[I_blk, :]
    d += 10 * 256;                    // Gy, H, Gs, Ls, LiT (16 x 17), Gam, Gam2, TA, statistics
    d += 4 * 256;                     // MFMA scratch
    d += 64;                          // reduction buffer
    return d * sizeof(double) + 96 * sizeof(int);
}

template <typename T>
__global__ __launch_bounds__(256) void csvd_kernel(CsvdArgs a) {
    typedef typename FactorOf<T>::type F;
    if (blockIdx.x % a.xs) return;
    extern __shared__ double smem[];
    const int tid = threadIdx.x, l64 = tid & 63, w4 = wave_id();
    const int wg = blockIdx.x / a.xs, G = a.G;
#ifdef IRCUR_PHASE_PROFILE
    uint64_t t_prev = __builtin_amdgcn_s_memrealtime();
    const uint64_t c_start = __builtin_amdgcn_s_memtime(), r_start = t_prev;
    uint64_t ph_[16];
    int ntest_ = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) ph_[i] = 0;
#define QADD(q) do { ph_[13] += (q).g; ph_[14] += (q).c; ph_[15] += (q).x; } while (0)
#else
#define QADD(q) do { (void)(q); } while (0)
#endif
    const int sI = a.sI, sJ = a.sJ, r = a.r, R = a.R;
    const int sJ16 = ((sJ + 15) / 16) * 16;
    const int KS = sJ16 / 4;             // k-steps of M_blk X
    const int ntj = sJ16 / 16;           // row tiles of Z
    const int tpg = (ntj + G - 1) / G;   // Z tiles per workgroup
    const int t0 = wg * tpg;             // first tile of this workgroup's slice
    const int ntl = max(0, min(tpg, ntj - t0));   // its tiles
    const int a0 = wg * 16;
    const int nb = max(0, min(16, sI - a0));
    const int live = min(16, sJ);         // columns of the block with a direction to hold
    const int64_t n1 = a.n1, n2 = a.n2;
    const int fd = sizeof(F) == 8 ? 0 : 1;

    double* Mb = smem;                    // 16 x sJ16 at mb_index(row, col)
    double* X = Mb + 17 * sJ16;           // sJ16 x 16, row stride XS
    double* Xp = X + sJ16 * XS;           // tpg x 256: X_{j-1} on the slice
    double* Zs = Xp + tpg * 256;          // tpg x 256: reduced Z on the slice
    double* Bsl = Zs + tpg * 256;         // tpg x 256: B_k[c, J_b] at [b_local * 16 + c]
    double* Y = Bsl + tpg * 256;          // 16 x 16
    double* Ab = Y + 256;                 // 16 x 16
    double* Gy = Ab + 256;                // small matrices: 10 x 256 doubles
    double* H = Gy + 256;
    double* Gs = H + 256;                 // 16 x XS
    double* Ls = Gs + 16 * XS;            // 16 x XS
    double* LiT = Ls + 16 * XS;           // 16 x XS
    double* Gam = LiT + 16 * XS;
    double* Gam2 = Gam + 256;
    double* TA = Gam2 + 256;
    double* cst = TA + 256;               // 16: Cholesky statistics
    double* scr = Gy + 10 * 256;          // 4 x 256
    double* red = scr + 4 * 256;          // 64
    int* dead = (int*)(red + 64);         // 64
    int* Il = dead + 64;                  // 16
    int* spare = Il + 16;                 // 16
    (void)spare;

    int32_t kd0;                          // run state: completed iterations, last e
    double el0;
    // ---- load: the core launch's M block (row-tiled layout), A_k[I_blk, :] and the
    // starting block X0 (one round trip; the core launch gathered and
    // thresholded the block on every compute unit).  X0: the previous basis
    // (warm == 1), else B_k[:, J]^T (warm == 2) or nothing (warm == 0) in the
    // wanted columns and pseudo-random entries in the others ----
    {
        const double* __restrict__ src = a.MA + (size_t)wg * KS * 64;   // row tile wg: KS blocks of 64
        constexpr int UL = 32;            // doubles per thread (|J| <= 512)
        double mv[UL];
#pragma unroll
        for (int u = 0; u < UL; ++u) mv[u] = src[min(tid + NT * u, KS * 64 - 1)];   // (clamped: no branch per load)
        const double av = a.Abc[(size_t)(a0 + (tid >> 4)) * 16 + (tid & 15)];
        // previous basis (row-major, 16 per row): entries tid + NT u in order;
        // B_k[:, J] (16 x sJ16): rows b = tid, tid + NT of each column, every
        // load in bounds and coalesced (|J| <= 512)
        const bool prev = a.warm == 1;
        double wv[2][16];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int h = u >> 4, c = u & 15;
            const int i = prev ? min(tid + NT * u, 16 * sJ16 - 1)
                               : (c < r ? c : 0) * sJ16 + min(tid + NT * h, sJ16 - 1);
            wv[h][c] = (prev || a.warm == 2) ? (prev ? a.prevV : a.Bsc)[i] : 0.0;
        }
        // the run state is read with the loads above in flight; a stopped run
        // returns before it writes anything
        kd0 = a.st->k_done;
        el0 = a.st->e_last;
        if (a.st->stop) return;
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const int e = tid + NT * u;
            if (e < KS * 64) {
                const int ks = e >> 6, l = e & 63;
                Mb[mb_index(l & 15, 4 * ks + (l >> 4))] = mv[u];
            }
        }
        Ab[tid] = (tid >> 4) < nb ? av : 0.0;
        // the starting block: rows past |J| and columns past `live` zero; the
        // wanted columns (warm 2) or all of them (warm 1) from the loads; the
        // other entries pseudo-random, filled below
        if (prev) {
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const int e = tid + NT * u, b = e >> 4, c = e & 15;
                if (e < 16 * sJ16) X[b * XS + c] = (b < sJ && c < live) ? wv[u >> 4][u & 15] : 0.0;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const int h = u >> 4, c = u & 15, b = tid + NT * h;
                if (b < sJ16) X[b * XS + c] = (b < sJ && c < live && c < r) ? wv[h][c] : 0.0;
            }
            const int c0 = a.warm == 2 ? r : 0;
#pragma unroll 1
            for (int c = c0; c < live; ++c)
                for (int b = tid; b < sJ; b += NT) X[b * XS + c] = rnd_x0(a.salt, b * 16 + c);
        }
        // B_k[:, J_b] of this workgroup's slice rows (epilogue, Gamma')
        for (int e = tid; e < ntl * 256; e += NT) {
            const int b = 16 * t0 + (e >> 4), c = e & 15;
            Bsl[e] = a.Bsc[(size_t)c * sJ16 + b];
        }
    }
    __syncthreads();
    // a single Cholesky QR pass keeps X^T X within about 16 eps kappa^2 of I
    const double tol_k = a.tol_e > 0.0 ? fmax(a.tol, a.tol_e * (kd0 > 0 ? el0 : 1.0)) : a.tol;
    const double kappa2_one = 0.01 * tol_k / (16.0 * 2.220446049250313e-16);
    const int min_passes = 1;
    CPHASE(0);
    // the previous basis is tested as it stands (after one Cholesky QR pass:
    // its columns are orthonormal to within the previous launch's tolerance);
    // the other starting blocks are not orthonormal and never pass a test, so
    // their first product with M^T M is a plain power step and the Cholesky
    // QR that follows it orthonormalises M^T M X0 (the span that the power
    // step from an orthonormalised X0 would reach)
    if (a.warm == 1) {
        const QTimes q = cholqr(X, sJ16, sJ, live, r, kappa2_one, min_passes, Gs, LiT, dead, cst, scr, a.salt + 17);
        QADD(q);
    }
    CPHASE(1);

    // ---- subspace iteration -------------------------------------------------
    double* Zp = a.Zp + (size_t)wg * sJ16 * 16;
    double* Gp = a.Gp + (size_t)wg * 768;
    uint32_t nbar = 0;
    int it = 0;                 // applications of A = M^T M
    bool test = a.warm == 1;    // this application tests Q (X orthonormal)
    bool power = true;          // the current sweep uses scaled power steps
    bool last_power = true;     // ... and the sweep before it
    double rate = 1.0;          // per-degree residual factor expected of the sweep
    double spread = 1.0;        // per-degree growth of the largest over the smallest wanted quotient
    int m = 1, j = 0;           // sweep degree, filter steps done in the sweep
    double cs = 0.0, es = 0.0, sg1 = 0.0, sg = 0.0, scale = 1.0;
    double res = 0.0, res_sweep = -1.0;
    bool conv = false;
    double widen = 1.0;         // filter interval [0, b]: b = 1.02 widen bx (the extra columns'
                                // quotients estimate sigma_{r+1}^2 from below)
    int cool = 0;               // tests whose sweep uses power steps (after a sweep that fell short)
    double bx_prev = -1.0;      // extra columns' largest quotient at the previous test
    double pred = 1.0;          // residual factor predicted for the current sweep
    double hi_t = 0.0, lo_t = 0.0;   // largest and smallest wanted quotients at the last test
    for (;;) {
        // Y = M_blk X: wave w takes the k-steps w, w + 4, ... (ntj of them), the
        // operands of each pair requested before the products of the pair
        // before; the four partial tiles summed in wave order.  Every wave ends
        // with Y in the B-operand layout, yb[ks] = Y[4 ks + l/16][l % 16].
        double yb[4];
        {
            constexpr int ST = 272;           // 4 k-steps further on, in both layouts
            const ldouble* mp = lp(Mb) + w4 * 68 + (l64 >> 4) * 17 + (l64 & 15);
            const ldouble* xp = lp(X) + (4 * w4 + (l64 >> 4)) * XS + (l64 & 15);
            const int n = ntj;
            d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
            double a0 = mp[0], b0 = xp[0], a1 = mp[min(1, n - 1) * ST], b1 = xp[min(1, n - 1) * ST];
            for (int u = 0; u < n; u += 2) {
                const int u2 = min(u + 2, n - 1), u3 = min(u + 3, n - 1);
                const double na0 = mp[u2 * ST], nb0 = xp[u2 * ST], na1 = mp[u3 * ST], nb1 = xp[u3 * ST];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
                acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(u + 1 < n ? a1 : 0.0, b1, acc2, 0, 0, 0);
                a0 = na0; b0 = nb0; a1 = na1; b1 = nb1;
            }
            acc += acc2;
            ldouble* sc = lp(scr);
#pragma unroll
            for (int v = 0; v < 4; ++v) sc[w4 * 256 + ((l64 >> 4) + 4 * v) * 16 + (l64 & 15)] = acc[v];
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int e = (4 * ks + (l64 >> 4)) * 16 + (l64 & 15);
                yb[ks] = ((sc[e] + sc[256 + e]) + sc[512 + e]) + sc[768 + e];
            }
            if (w4 == 0) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) lp(Y)[(4 * ks + (l64 >> 4)) * 16 + (l64 & 15)] = yb[ks];
            }
        }
        CPHASE(2);
        // partial Z_g = M_blk^T Y (tile-lane order), wave w taking the tiles
        // w, w + 4, ... two at a time; on a test also the partial Grams Y^T Y,
        // Y^T A_blk and Gamma'_g = B_k[:, J_slice] X_slice
        {
            const ldouble* mc = lp(Mb) + mb_index(l64 >> 4, l64 & 15);
            for (int tj = w4; tj < ntj; tj += 8) {
                const int tk = tj + 4;
                const bool two = tk < ntj;
                double av[4], cv[4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    av[ks] = mc[tj * 272 + 4 * ks];
                    cv[ks] = mc[(two ? tk : tj) * 272 + 4 * ks];
                }
                d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
                if (two) {
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], yb[ks], acc, 0, 0, 0);
                        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(cv[ks], yb[ks], acc2, 0, 0, 0);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        st_dev(Zp + (size_t)tj * 256 + v * 64 + l64, acc[v]);
                        st_dev(Zp + (size_t)tk * 256 + v * 64 + l64, acc2[v]);
                    }
                } else {
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], yb[ks], acc, 0, 0, 0);
#pragma unroll
                    for (int v = 0; v < 4; ++v) st_dev(Zp + (size_t)tj * 256 + v * 64 + l64, acc[v]);
                }
            }
        }
        if (test && w4 < 3) {
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            if (w4 == 0) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(yb[ks], yb[ks], acc, 0, 0, 0);
            } else if (w4 == 1) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(yb[ks], Ab[(4 * ks + (l64 >> 4)) * 16 + (l64 & 15)], acc,
                                                               0, 0, 0);
            } else {
                for (int q = 0; q < ntl; ++q)
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int bl = 4 * ks + (l64 >> 4);
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Bsl[q * 256 + bl * 16 + (l64 & 15)],
                                                                   X[(16 * (t0 + q) + bl) * XS + (l64 & 15)], acc, 0, 0, 0);
                    }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) st_dev(Gp + w4 * 256 + v * 64 + l64, acc[v]);
        }
        CPHASE(3);
        ++nbar;
        grid_sync(&a.st->bar_ctr, nbar * (uint32_t)G, &a.st->svd_fail);
        CPHASE(4);
        // reduce: Gy (test) in full and this workgroup's row tiles of Z, the
        // loads of Gy and of the first tile in one batch
        {
            const int ix = ((tid & 63) >> 4) * 16 + 64 * (tid >> 6) + (tid & 15);
            if (test && ntl >= 1) {
                double g, z;
                sum_parts2(a.Gp + tid, 768, a.Zp + (size_t)t0 * 256 + tid, (size_t)sJ16 * 16, G, g, z);
                Gy[ix] = g;
                Zs[ix] = z;
            } else {
                if (test) Gy[ix] = sum_parts(a.Gp + tid, 768, G);
                if (ntl >= 1) Zs[ix] = sum_parts(a.Zp + (size_t)t0 * 256 + tid, (size_t)sJ16 * 16, G);
            }
            for (int q = 1; q < ntl; ++q) Zs[q * 256 + ix] = sum_parts(a.Zp + (size_t)(t0 + q) * 256 + tid, (size_t)sJ16 * 16, G);
        }
        __syncthreads();
        CPHASE(5);
        if (test) {
            // filter of the sweep from the Rayleigh quotients of the columns of Q:
            // wanted columns in [lo, hi], extra ones below bx (~ sigma_{r+1}^2)
            double hi = 0.0, lo = 0.0, bx = 0.0;
            {
                double dg[16];
#pragma unroll
                for (int c = 0; c < 16; ++c) dg[c] = Gy[c * 17];
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    if (c < r) { hi = fmax(hi, dg[c]); lo = c == 0 ? dg[c] : fmin(lo, dg[c]); }
                    else if (c < live) bx = fmax(bx, dg[c]);
                }
            }
            hi_t = hi;
            lo_t = lo;
            last_power = power;
            // Chebyshev only once the extra columns' estimate of sigma_{r+1}^2 has
            // settled (2% between tests) and lies clearly below the wanted ones
            const bool stable = bx_prev > 0.0 && fabs(bx - bx_prev) <= 0.02 * bx;
            bx_prev = bx;
            power = cool > 0 || !(bx > 0.0) || !(bx < 0.9 * lo) || !stable;
            if (cool > 0) --cool;
            if (power) {
                cs = 0.0; es = 0.0;
                scale = hi > 0.0 ? 1.0 / hi : 1.0;
            } else {
                const double bb = fmin(1.02 * widen * bx, 0.95 * lo);
                cs = 0.5 * bb; es = 0.5 * bb;
                sg1 = es / (hi - cs);
                sg = sg1;
                scale = sg1 / es;
                // per-degree rate of the filter at the smallest wanted quotient,
                // and the per-degree spread between the largest and smallest
                // wanted ones (it costs the smaller wanted directions digits
                // in the Cholesky QR that follows the sweep)
                const double xr = (lo - cs) / es, xh = (hi - cs) / es;
                const double glo = xr + __builtin_sqrt(fmax(xr * xr - 1.0, 0.0));
                const double ghi = xh + __builtin_sqrt(fmax(xh * xh - 1.0, 0.0));
                rate = 1.0 / glo;
                spread = ghi / glo;
            }
            // residual of the first r columns over this workgroup's rows of Z
            double part = 0.0;
            for (int q = 0; q < ntl; ++q) {
                const int b = 16 * (t0 + q) + (tid >> 4), c = tid & 15;
                if (b < sJ && c < r) {
                    double xr_[16], gc_[16];
#pragma unroll
                    for (int d = 0; d < 16; ++d) { xr_[d] = X[b * XS + d]; gc_[d] = Gy[d * 16 + c]; }
                    double s = Zs[q * 256 + tid];
#pragma unroll
                    for (int d = 0; d < 16; ++d)
                        if (d < r) s = __builtin_fma(-xr_[d], gc_[d], s);
                    part = __builtin_fma(s, s, part);
                }
            }
            part = block_sum_dpp(part, red);
            if (tid == 0) st_dev(a.rp + wg, part);
        }
        // this workgroup's rows of the next block
        double sgn = 0.0;
        if (!test && !power) sgn = 1.0 / (2.0 / sg1 - sg);
        for (int q = 0; q < ntl; ++q) {
            const int e = q * 256 + tid, b = 16 * (t0 + q) + (tid >> 4);
            const double xj = X[b * XS + (tid & 15)];
            double xn;
            if (test || power) xn = (Zs[e] - cs * xj) * scale;
            else xn = (Zs[e] - cs * xj) * (2.0 * sgn / es) - (sg * sgn) * Xp[e];
            Xp[e] = xj;
            st_dev(a.Xr + (size_t)b * 16 + (tid & 15), b < sJ ? xn : 0.0);
        }
        if (!test && !power) sg = sgn;
        CPHASE(6);
        ++nbar;
        grid_sync(&a.st->bar_ctr, nbar * (uint32_t)G, &a.st->svd_fail);
        CPHASE(7);
        ++it;
        if (test) {
            double pn = 0.0;
            for (int g = tid; g < G; g += NT) pn += ld_dev(a.rp + g);
            // invariance residual of the wanted columns against the smallest
            // wanted quotient (~ sigma_r^2), with a floor at the rounding of
            // M^T M X (~ eps sigma_1^2)
            const double num = __builtin_sqrt(block_sum_dpp(pn, red));
            const double thr = fmax(tol_k * lo_t, 256.0 * 2.220446049250313e-16 * hi_t);
            res = lo_t > 0.0 ? num / lo_t : (num > 0.0 ? 1.0 : 0.0);
            conv = !(num > thr);
#ifdef IRCUR_PHASE_PROFILE
            // first launch of a run: the first eight tests (residual, applications, mode)
            if (wg == 0 && tid == 0 && a.st->k_done == 0 && !a.prof_slot && ntest_ < 8) {
                a.st->phase2[2 * ntest_] = __builtin_bit_cast(uint64_t, res);
                a.st->phase2[2 * ntest_ + 1] = (uint64_t)(it * 1000 + m * 10 + (power ? 1 : 0));
            }
            ++ntest_;
#endif
            if (conv || it >= a.max_it) break;        // X still holds the tested Q
            // a Chebyshev sweep that did not halve the residual: plain steps next
            // a Chebyshev sweep that did not reach the square root of its
            // predicted factor: the interval was too narrow (sigma_{r+1}^2
            // above b); one power step, then a wider interval
            if (!last_power && res_sweep > 0.0 && res > res_sweep * __builtin_sqrt(pred)) {
                widen *= 1.05;
                cool = 1;
            }
            res_sweep = res;
            // degree of the sweep: enough for the residual to reach tol at `rate`
            m = 1;
            if (!power) {
                m = 8;
                if (rate > 0.0 && rate < 1.0) m = (int)ceil(log(num / thr) / -log(rate));
                // a sweep of degree m loses about eps res spread^m in the wanted
                // directions: keep that a tenth of the tolerance
                if (spread > 1.0) {
                    const double room = 0.1 * tol_k / (2.220446049250313e-16 * fmax(res, 2.220446049250313e-16));
                    const int mmax = room > 1.0 ? (int)floor(log(room) / log(spread)) : 1;
                    m = min(m, max(1, mmax));
                }
                m = max(1, min(m, 8));
            }
            m = min(m, a.max_it - it);
            pred = power ? 1.0 : pow(rate, (double)m);
            j = 1;
        } else {
            ++j;
        }
        // all-gather the next block (one batch of loads per thread)
        {
            constexpr int B = 20;
            const int tot = sJ16 * 16;
            for (int e0 = tid; e0 < tot; e0 += NT * B) {
                double v[B];
#pragma unroll
                for (int u = 0; u < B; ++u) v[u] = e0 + u * NT < tot ? ld_dev(a.Xr + e0 + u * NT) : 0.0;
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int e = e0 + u * NT;
                    if (e < tot) X[(e >> 4) * XS + (e & 15)] = v[u];
                }
            }
        }
        __syncthreads();
        CPHASE(8);
        if (j >= m) {
            const QTimes q = cholqr(X, sJ16, sJ, live, r, kappa2_one, min_passes, Gs, LiT, dead, cst, scr,
                                    a.salt ^ (0x2545F4914F6CDD1Dull * (uint64_t)(it + 1)));
            QADD(q);
            test = true;
        } else {
            test = false;
        }
        CPHASE(9);
    }
    CPHASE(8);
    // no barrier follows: the last workgroup out returns both counters to zero
    // for the next launch
    if (tid == 0) {
        const uint32_t out = __hip_atomic_fetch_add(&a.st->bar_exit, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (out == (uint32_t)G - 1) {
            __hip_atomic_store(&a.st->bar_ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.st->bar_exit, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // ---- epilogue -------------------------------------------------------------
    double bx = 0.0;
    {
        double dg[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) dg[c] = Gy[c * 17];
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c >= r && c < live) bx = fmax(bx, dg[c]);
    }
    // wave 0: Gy_rr = Ly Ly^T; a pivot <= s eps max_j Gy_jj is a direction the
    // Gram matrix cannot resolve (sigma below about sqrt(s eps) sigma_1):
    // dropped.  Waves 1-3 meanwhile: H = Y^T A_blk and Gamma' = B_k[:, J] Q from
    // the partials of the last test (columns >= r of Gamma' zero), the next
    // starting basis (all columns of this slice's rows), and the columns >= r
    // of the slice rows of X zeroed (the outputs use the first r)
    const double ptol = (double)(sI > sJ ? sI : sJ) * 2.220446049250313e-16;
    chol16(Gy, 16, r, ptol, false, Ls, LiT, dead, nullptr, scr, 16, false);
    if (w4 != 0) {
        for (int e = tid - 64; e < 256; e += NT - 64) {
            const int ix = ((e & 63) >> 4) * 16 + 64 * (e >> 6) + (e & 15);
            double h, g2;
            sum_parts2(a.Gp + 256 + e, 768, a.Gp + 512 + e, 768, G, h, g2);
            H[ix] = h;
            Gam2[ix] = (ix & 15) >= r ? 0.0 : g2;
        }
        for (int e = tid - 64; e < ntl * 256; e += NT - 64) {
            const int b = 16 * t0 + (e >> 4), c = e & 15;
            a.prevV[b * 16 + c] = X[b * XS + c];
            if (c >= r) X[b * XS + c] = 0.0;
        }
    }
    __syncthreads();
    // Wt_blk = Y Ly^-T, Gamma = Ly^-1 H, TA = Ly^-T
    double* Wb = Gs;
    if (w4 == 0) {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Y[(l64 & 15) * 16 + 4 * ks + (l64 >> 4)],
                                                       LiT[(4 * ks + (l64 >> 4)) * XS + (l64 & 15)], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = (l64 >> 4) + 4 * v;
            Wb[row * 16 + (l64 & 15)] = row < nb ? acc[v] : 0.0;
        }
    }
    {
        const int i = tid >> 4, jj = tid & 15;
        double li_[16], h_[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) { li_[k] = LiT[k * XS + i]; h_[k] = H[k * 16 + jj]; }
        double g = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) g = __builtin_fma(li_[k], h_[k], g);
        Gam[tid] = g;
        TA[tid] = LiT[i * XS + jj];
    }
    __syncthreads();
    // Delta_blk = A_blk - Wt_blk Gamma (Wt_blk Gamma into Y)
    if (w4 == 0) {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Wb[(l64 & 15) * 16 + 4 * ks + (l64 >> 4)],
                                                       Gam[(4 * ks + (l64 >> 4)) * 16 + (l64 & 15)], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) Y[((l64 >> 4) + 4 * v) * 16 + (l64 & 15)] = acc[v];
    }
    __syncthreads();
    for (int e = tid; e < nb * R; e += NT) {
        const int ar = e / R, c = e - ar * R;
        if (a.rowI) {                                      // (the vector pass's row form)
            const int64_t base = (int64_t)(a0 + ar) * a.qs;
            fput(a.rowI, base + c, Ab[ar * 16 + c], fd);
            fput(a.rowI, base + R + c, Wb[ar * 16 + c], fd);
            fput(a.rowI, base + 2 * R + c, Ab[ar * 16 + c] - Y[ar * 16 + c], fd);
        }
        a.W[(int64_t)(a0 + ar) * R + c] = Wb[ar * 16 + c];
    }
    // rows of this workgroup's slice: [B_k[:, J_b] | Q[b, :] | B_k[:, J_b] - Gamma' Q[b, :]^T],
    // the last part formed first into Zs (no longer needed), zero past |J|
    for (int e = tid; e < ntl * 256; e += NT) {
        const int bl = e >> 4, c = e & 15;
        const int b = 16 * t0 + bl;
        double dl = 0.0;
        if (b < sJ && c < R) {
            double g_[16], x_[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) { g_[i] = Gam2[c * 16 + i]; x_[i] = X[b * XS + i]; }
            double sg = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) sg = __builtin_fma(g_[i], x_[i], sg);
            dl = Bsl[e] - sg;
        }
        Zs[e] = dl;
    }
    __syncthreads();
    for (int e = tid; e < ntl * 16 * R; e += NT) {
        const int bl = e / R, c = e - bl * R;
        const int b = 16 * t0 + bl;
        if (b >= sJ) continue;
        if (a.rowJ) {
            const int64_t base = (int64_t)b * a.qs;
            fput(a.rowJ, base + c, Bsl[bl * 16 + c], fd);
            fput(a.rowJ, base + R + c, X[b * XS + c], fd);
            fput(a.rowJ, base + 2 * R + c, Zs[bl * 16 + c], fd);
        }
        a.V[(int64_t)b * R + c] = X[b * XS + c];
    }
    // the same per-row data in the operand-tile order of the matrix-core pass:
    // per 16-row tile, ceil(R/4) blocks of the A operand of the products with
    // the factor (lane l: row l % 16, factor index 4 ks + l / 16), as many of
    // the Delta part, then four blocks of the projection part (lane l: row of
    // accumulator register v in the pass's layout, factor index l % 16)
    if (a.rowIt) {
        const int KRt = (R + 3) / 4, NBt = (2 * KRt + 4) * 64;
        for (int e = tid; e < (1 + ntl) * NBt; e += NT) {
            const int q = e / NBt - 1, f = e - (q + 1) * NBt, kind = f >> 6, l = f & 63;
            double v = 0.0;
            int row, c;
            if (kind < 2 * KRt) {
                row = l & 15;
                c = 4 * (kind < KRt ? kind : kind - KRt) + (l >> 4);
            } else {
                const int vv = kind - 2 * KRt;
                row = fd == 0 ? (l >> 4) + 4 * vv : 4 * (l >> 4) + vv;
                c = l & 15;
            }
            if (q < 0) {                             // this workgroup's row tile of I
                if (row < nb && c < R)
                    v = kind < KRt ? Ab[row * 16 + c]
                                   : (kind < 2 * KRt ? Ab[row * 16 + c] - Y[row * 16 + c] : Wb[row * 16 + c]);
                fput(a.rowIt, (int64_t)wg * NBt + f, v, fd);
            } else {                                 // slice tile t0 + q of J
                const int b = 16 * (t0 + q) + row;
                if (b < sJ && c < R)
                    v = kind < KRt ? Bsl[q * 256 + row * 16 + c]
                                   : (kind < 2 * KRt ? Zs[q * 256 + row * 16 + c] : X[b * XS + c]);
                fput(a.rowJt, (int64_t)(t0 + q) * NBt + f, v, fd);
            }
        }
    }
    if (wg == 0) {
        for (int e = tid; e < R * R; e += NT) {
            const int c = e / R, d = e - c * R;
            fput(a.GmI, e, Gam[c * 16 + d], fd);
            fput(a.GmJ, e, Gam2[d * 16 + c], fd);
            fput(a.scaleJ, e, TA[c * 16 + d], fd);
            a.TAd[e] = TA[c * 16 + d];
            a.sigma[e] = Ls[d * XS + c];                               // Kc = Ly^T: H_r(M) = Wt Kc Q^T
        }
        if (tid == 0) {
            int kept = 0, dd[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) dd[i] = dead[i];
#pragma unroll
            for (int i = 0; i < 16; ++i) kept += (i < r && dd[i] == 0) ? 1 : 0;
            a.info->iters = it;
            a.info->kept = kept;
            a.info->resid = res;
            a.info->bx = live > r ? bx : -1.0;          // (the gap: the finalize launch)
            a.info->gap = -1.0;
            if (!conv) a.st->svd_capped = 1;
            if (kept < r && Gy[0] > 0.0) a.st->rank_drop = 1;
        }
    }
    CPHASE(10);
#ifdef IRCUR_PHASE_PROFILE
    if (wg == 0 && tid == 0) {
        uint64_t* dst = a.prof_slot ? a.st->phase2 : a.st->phase;
        for (int i = 0; i < 16; ++i) dst[i] += ph_[i];
        (void)c_start; (void)r_start;
    }
#endif
}

hipError_t launch_csvd(const CsvdArgs& a, int dtype, size_t lds_bytes, hipStream_t s) {
    const void* fn = nullptr;
    int slot = -1;
    if (dtype == 0) { fn = (const void*)csvd_kernel<double>; slot = 0; }
    if (dtype == 1) { fn = (const void*)csvd_kernel<float>; slot = 1; }
    if (dtype == 2) { fn = (const void*)csvd_kernel<bf16_t>; slot = 2; }
    if (!fn || a.G < 1 || a.R > 16 || a.xs < 1) return hipErrorInvalidValue;
    static bool attr_set[3] = {false, false, false};
    if (!attr_set[slot]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set[slot] = true;
    }
    CsvdArgs b = a;
    void* args[] = {&b};
    return hipLaunchKernel(fn, dim3(a.G * a.xs), dim3(NT), args, lds_bytes, s);
}

}  // namespace ircur
