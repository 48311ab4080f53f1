// Host runtime and C ABI of libircur (see include/ircur.h).
//
// One IRCUR iteration (Algorithm 1, k -> k+1) is four launches on the
// context's stream:
//   core      M = [D - S_{k+1}]_{I,J}                      (Phase I, eq. (4), (5))
//   svd       top-r SVD of M, pinv rule, per-row data of the pass (Phase II)
//   pass      B_{k+1} = W_r^T R, A_{k+1} = C V_r Sigma_r^+ and the partial
//             sums of e_{k+1}                             (eq. (2), (3), (6))
//   finalize  e_{k+1}, history, device-side stop flag
// Iterations are enqueued in chunks; every kernel returns at once when the
// stop flag is set, so the host reads back state once per chunk.
#include "ircur_internal.h"
#include "../../include/ircur.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace ircur;

// --------------------------------------------------------------- sampler ---
// SplitMix64 (Steele, Lea, Flood 2014), Floyd's sampling, multiply-shift.
namespace {

inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct SplitMix64 {
    uint64_t state;
    uint64_t next() {
        state += 0x9E3779B97F4A7C15ull;
        return sm_mix(state);
    }
    uint64_t below(uint64_t m) {   // uniform in [0, m)
        return (uint64_t)(((unsigned __int128)next() * (unsigned __int128)m) >> 64);
    }
};

SplitMix64 index_stream(uint64_t seed, int64_t t) {
    const uint64_t key = seed ^ ((uint64_t)(t + 1) * 0xD1B54A32D192ED03ull);
    return SplitMix64{sm_mix(key)};
}

// k distinct values of [0, n), ascending (Floyd's algorithm).  Membership is
// a bitmap over [0, n) (cleared per call), so a draw costs O(k + n/64).
void floyd(SplitMix64& g, int64_t n, int32_t k, int32_t* out) {
    static thread_local std::vector<uint64_t> bits;
    const size_t words = (size_t)((n + 63) / 64);
    bits.assign(words, 0ull);
    for (int64_t j = n - k; j < n; ++j) {
        const int64_t t = (int64_t)g.below((uint64_t)(j + 1));
        uint64_t& w = bits[(size_t)(t >> 6)];
        const uint64_t m = 1ull << (t & 63);
        if (w & m) bits[(size_t)(j >> 6)] |= 1ull << (j & 63);
        else w |= m;
    }
    int32_t o = 0;
    for (size_t wi = 0; wi < words && o < k; ++wi) {
        uint64_t w = bits[wi];
        while (w) {
            const int b = __builtin_ctzll(w);
            out[o++] = (int32_t)(wi * 64 + b);
            w &= w - 1;
        }
    }
}

constexpr int kChunk = 32;        // iterations per enqueue batch
constexpr int kRing = 2 * kChunk; // index-set slots: two batches in flight

float round_down_float(double z) {
    if (!(z < 3.4e38)) return INFINITY;
    float f = (float)z;
    if ((double)f > z) f = std::nextafter(f, -INFINITY);
    return f;
}

}  // namespace

// ------------------------------------------------ fixed device workspace ---
// The workspace of ircur_to_svd_noalloc, for callers that cannot allocate:
// Algorithm 2's Gram partials (2 sides x at most 256 workgroups x R x R) and
// its two pairs of R x R maps, R <= IRCUR_MAX_RANK: 528384 doubles, 4.03 MiB.
// Every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` only stands for the symbol: its device address is
// taken once per device with hipGetSymbolAddress (at ircur_init, with that
// device current) and only that address is handed to kernels.
namespace {
constexpr size_t kScratchDoubles = 2 * 256 * (size_t)IRCUR_MAX_RANK * IRCUR_MAX_RANK
                                   + 4 * (size_t)IRCUR_MAX_RANK * IRCUR_MAX_RANK;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Looks up (once per device; the device must be current) and returns the
// device address of `scratch`; nullptr when the lookup fails.
double* noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_dev[device] = (double*)ptr;
    }
    return g_scratch_dev[device];
}

double* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}

// Workgroups per side of Algorithm 2's Gram kernel and the workspace it needs.
int alg2_groups(const ircur_params& p) {
    return (int)std::min<int64_t>(256, (std::max(p.n1, p.n2) + 127) / 128);
}
size_t alg2_doubles(int nwg, size_t R) { return 2 * (size_t)nwg * R * R + 4 * R * R; }

}  // namespace

// --------------------------------------------------------------- context ---

struct ircur_ctx {
    ircur_params p{};
    int R = 0, psvd = 0, G = 0, bs = 0;
    size_t svd_lds = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    const void* D = nullptr;
    const void* Dt = nullptr;
    int64_t ldDt = 0;
    void* Dt_own = nullptr;
    size_t esz = 0, fsz = 0;
    void* At[2] = {nullptr, nullptr};
    void* B[2] = {nullptr, nullptr};
    // index sets of the ring's slots, I then J in each slot (one upload per batch)
    int32_t* IJdev = nullptr;
    int32_t* IJpin = nullptr;
    double* M = nullptr;
    double* MA = nullptr;
    double* MB = nullptr;
    double* Zp = nullptr;
    double* Gp = nullptr;
    double* prevV = nullptr;
    double* W = nullptr;
    double* V = nullptr;
    double* sigma = nullptr;
    void* rowI = nullptr;
    void* rowJ = nullptr;
    void* GmI = nullptr;
    void* GmJ = nullptr;
    void* scaleJ = nullptr;
    double* TAd = nullptr;
    double* Abc = nullptr;          // compact A_k[I, :] (sI16 x 16), written by the core kernel
    double* Bsc = nullptr;          // compact B_k[:, J] (16 x sJ16)
    double* Zr = nullptr;           // reduced Z of the SVD (sJ16 x 16)
    double* rp = nullptr;           // SVD residual parts (G)
    bool lds_svd = false;           // the SVD keeps its block of M in LDS (P = 16)
    bool csvd = false;              // core gather and SVD in one launch (ircur_csvd.hip)
    int Gc = 0;                     // its workgroups, ceil(sI / 16)
    int Xs = 1;                     // their stride in the grid (all on one XCD when it fits)
    bool p16 = false;               // the matrix-core pass (with the one-launch SVD's operand tiles)
    void* rowIt = nullptr;          // per-row data in operand-tile order, rows I and J
    void* rowJt = nullptr;
    size_t csvd_lds = 0;
    double* Xr = nullptr;           // its exchange block (sJ16 x 16)
    std::vector<double> zsched;     // the caller's threshold schedule (empty: geometric)
    int32_t* Icur = nullptr;        // index sets of an export (device)
    int32_t* Jcur = nullptr;
    unsigned long long* nnz = nullptr;
    double* alg2_buf = nullptr;     // Algorithm 2 workspace (allocated on first use)
    double* part_row = nullptr;
    double* part_col = nullptr;
    int nwg_row = 0, nwg_col = 0;
    int ns_row = 1, ns_col = 1;        // pass row blocks per column tile
    void* pacc = nullptr;              // pass partial sums of row-split tiles
    double* pzd = nullptr;
    uint32_t* pcnt = nullptr;          // per-tile tickets (zero between launches)
    DevState* st = nullptr;
    DevState* st_host = nullptr;   // pinned
    DevState* snap_host = nullptr; // pinned, 2: the state after each of two chunks in flight (solve)
    hipEvent_t snap_ev[2] = {nullptr, nullptr};
    SvdInfo* info = nullptr;       // max_iter records
    double* hist = nullptr;        // max_iter
    int32_t k = 0;                 // completed iterations (host view after sync)
    int32_t k_enq = 0;             // next iteration to enqueue
    int32_t k_base = 0;            // k at which the factors were last set from outside
    int32_t batch = 0;             // batches enqueued (selects the ring half)
    bool stopped = false;
    hipEvent_t h2d[2] = {nullptr, nullptr};
    bool h2d_pending[2] = {false, false};
    int32_t acc_next = 0;          // next iteration whose timing is not yet summed
    std::vector<int32_t> setsI, setsJ;   // per iteration, host copy
    std::vector<int32_t> lastJ;          // J of the previous svd (warm start)
    bool have_prevV = false;
    bool timing = false;
    hipEvent_t ev[kRing][5];
    bool ev_made = false;
    int32_t last_k = -1;                 // last enqueued iteration and its device index sets
    const int32_t* lastIdev = nullptr;
    const int32_t* lastJdev = nullptr;
    double tsum[4] = {0, 0, 0, 0};
    int64_t tcount = 0;
    std::string err;
};

namespace {

int fail(ircur_ctx* c, int code, const char* msg) {
    if (c) c->err = msg;
    return code;
}

#define TRY_ALLOC(ctx, x)            \
    do {                             \
        int r_ = (x);                \
        if (r_) return r_;           \
    } while (0)

#define HIPCHK(ctx, x)                                                        \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            if (ctx) (ctx)->err = std::string(#x) + ": " + hipGetErrorString(e_); \
            return IRCUR_ERR_DEVICE;                                          \
        }                                                                     \
    } while (0)

int validate(const ircur_params* p, const void* D, const void* Dt, int64_t ldDt) {
    if (!p || !D) return IRCUR_ERR_ARG;
    if (p->n1 < 1 || p->n2 < 1 || p->n1 > INT32_MAX || p->n2 > INT32_MAX) return IRCUR_ERR_ARG;
    if (p->ldD < p->n2) return IRCUR_ERR_ARG;
    if (p->sI < 1 || p->sJ < 1 || p->sI > p->n1 || p->sJ > p->n2) return IRCUR_ERR_ARG;
    if (p->r < 1 || p->r > IRCUR_MAX_RANK || p->r > p->sI || p->r > p->sJ) return IRCUR_ERR_ARG;
    if (p->dtype < 0 || p->dtype > 2) return IRCUR_ERR_ARG;
    if (p->resample != 0 && p->resample != 1) return IRCUR_ERR_ARG;
    if (p->err_mode != 0 && p->err_mode != 1) return IRCUR_ERR_ARG;
    if (!(p->zeta0 >= 0.0) || std::isnan(p->zeta0)) return IRCUR_ERR_ARG;
    if (!(p->gamma > 0.0 && p->gamma <= 1.0)) return IRCUR_ERR_ARG;
    if (std::isnan(p->eps)) return IRCUR_ERR_ARG;
    if (p->max_iter < 1) return IRCUR_ERR_ARG;
    if (!(p->svd_tol >= 0.0) || p->svd_max_it < 0) return IRCUR_ERR_ARG;
    if (p->svd_block != 0 &&
        (p->svd_block < p->r || p->svd_block > 32 || p->svd_block > p->sI || p->svd_block > p->sJ))
        return IRCUR_ERR_ARG;
    if (Dt && ldDt < p->n1) return IRCUR_ERR_ARG;
    if (p->zeta_sched)
        for (int32_t k = 0; k < p->max_iter; ++k)
            if (!(p->zeta_sched[k] >= 0.0) || std::isinf(p->zeta_sched[k])) return IRCUR_ERR_ARG;
    return IRCUR_OK;
}

template <typename T>
int dalloc(ircur_ctx* c, T** ptr, size_t count) {
    void* q = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
        *ptr = nullptr;
        c->err = "hipMalloc failed";
        return IRCUR_ERR_ALLOC;
    }
    *ptr = (T*)q;
    return IRCUR_OK;
}

int dalloc_bytes(ircur_ctx* c, void** ptr, size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (hipMalloc(ptr, bytes) != hipSuccess) {
        *ptr = nullptr;
        c->err = "hipMalloc failed";
        return IRCUR_ERR_ALLOC;
    }
    return IRCUR_OK;
}

void free_all(ircur_ctx* c) {
    void* bufs[] = {c->Dt_own, c->At[0], c->At[1], c->B[0], c->B[1], c->IJdev,
                    c->M, c->MA, c->MB, c->Zp, c->Gp, c->prevV, c->W, c->V, c->sigma, c->rowI,
                    c->rowJ, c->GmI, c->GmJ, c->scaleJ, c->TAd, c->Abc, c->Bsc, c->Zr, c->rp, c->Xr, c->Icur, c->Jcur, c->nnz, c->alg2_buf, c->part_row, c->part_col, c->pacc, c->pzd, c->pcnt, c->st,
                    c->info, c->hist, c->rowIt, c->rowJt};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (c->IJpin) (void)hipHostFree(c->IJpin);
    if (c->st_host) (void)hipHostFree(c->st_host);
    if (c->snap_host) (void)hipHostFree(c->snap_host);
    if (c->ev_made)
        for (int i = 0; i < kRing; ++i)
            for (int j = 0; j < 5; ++j) (void)hipEventDestroy(c->ev[i][j]);
    for (int h = 0; h < 2; ++h) {
        if (c->h2d[h]) (void)hipEventDestroy(c->h2d[h]);
        if (c->snap_ev[h]) (void)hipEventDestroy(c->snap_ev[h]);
    }
}

// zeta_{k+1} of Algorithm 1, Phase I: the caller's schedule, else gamma^k zeta_0.
double zeta_at(const ircur_ctx* c, int k) {
    if (!c->zsched.empty()) return c->zsched[std::min<size_t>((size_t)std::max(k, 0), c->zsched.size() - 1)];
    return c->p.zeta0 * std::pow(c->p.gamma, (double)k);
}

// Reset device state, factors and history to L_0 = 0, k = 0.
int reset_state(ircur_ctx* c) {
    const size_t fa = (size_t)c->R * c->p.n1 * c->fsz, fb = (size_t)c->R * c->p.n2 * c->fsz;
    for (int i = 0; i < 2; ++i) {
        HIPCHK(c, hipMemsetAsync(c->At[i], 0, fa, c->stream));
        HIPCHK(c, hipMemsetAsync(c->B[i], 0, fb, c->stream));
    }
    HIPCHK(c, hipMemsetAsync(c->st, 0, sizeof(DevState), c->stream));
    HIPCHK(c, hipMemsetAsync(c->hist, 0, sizeof(double) * c->p.max_iter, c->stream));
    HIPCHK(c, hipMemsetAsync(c->info, 0, sizeof(SvdInfo) * c->p.max_iter, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->k = 0;
    c->k_enq = 0;
    c->k_base = 0;
    c->acc_next = 0;
    c->stopped = false;
    c->have_prevV = false;
    c->last_k = -1;
    c->lastJ.clear();
    c->tsum[0] = c->tsum[1] = c->tsum[2] = c->tsum[3] = 0.0;
    c->tcount = 0;
    return IRCUR_OK;
}

// Sum the kernel times of iteration `it` (its events must have completed).
void accumulate_timing(ircur_ctx* c, int it) {
    const int slot = it % kRing;
    for (int q = 0; q < 4; ++q) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[slot][q], c->ev[slot][q + 1]) == hipSuccess) c->tsum[q] += ms;
    }
    c->tcount += 1;
}

int read_state(ircur_ctx* c) {
    HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->k = c->st_host->k_done;
    c->stopped = c->st_host->stop != 0;
    // every enqueued launch has finished: iterations past k were no-ops
    c->k_enq = c->k;
    if (c->timing && c->ev_made) {
        for (int it = c->acc_next; it < c->k; ++it) accumulate_timing(c, it);
        c->acc_next = c->k;
    }
    return IRCUR_OK;
}

int status_after(ircur_ctx* c) {
    if (c->st_host->svd_fail) return fail(c, IRCUR_ERR_SVD, "SVD grid barrier timed out");
    if (c->st_host->nonfinite) return fail(c, IRCUR_ERR_NONFINITE, "non-finite value in D or iterates");
    return IRCUR_OK;
}

// Arguments of the fused row/column pass of iteration k.
PassArgs pass_args(ircur_ctx* c, int k, const int32_t* Id, const int32_t* Jd) {
    const ircur_params& p = c->p;
    const int cur = k & 1, nxt = cur ^ 1;
    const double zeta = zeta_at(c, k);
    PassArgs pa{};
    SideArgs& r0 = pa.side[0];
    r0.X = c->D; r0.ldX = p.ldD; r0.rows = Id; r0.s = p.sI; r0.n = p.n2; r0.P = c->B[cur];
    r0.rowdata = c->rowI; r0.tiled = c->rowIt; r0.Gm = c->GmI; r0.outmat = nullptr; r0.out = c->B[nxt];
    r0.part = c->part_row; r0.nwg = c->nwg_row;
    const size_t fblk = pass_split_bytes(p.dtype, c->R) - 128 * sizeof(double);   // F sums per block
    r0.nsplit = c->ns_row; r0.pacc = c->pacc; r0.pzd = c->pzd; r0.cnt = c->pcnt;
    SideArgs& r1 = pa.side[1];
    r1.X = c->Dt; r1.ldX = c->ldDt; r1.rows = Jd; r1.s = p.sJ; r1.n = p.n1; r1.P = c->At[cur];
    r1.rowdata = c->rowJ; r1.tiled = c->rowJt; r1.Gm = c->GmJ; r1.outmat = c->scaleJ; r1.out = c->At[nxt];
    r1.part = c->part_col; r1.nwg = c->nwg_col;
    const size_t nb0 = (size_t)c->nwg_row * c->ns_row;
    r1.nsplit = c->ns_col; r1.pacc = (char*)c->pacc + nb0 * fblk; r1.pzd = c->pzd + nb0 * 128;
    r1.cnt = c->pcnt + c->nwg_row;
    pa.zeta = zeta; pa.zeta_f = round_down_float(zeta); pa.err_mode = p.err_mode; pa.st = c->st;
    return pa;
}

// Enqueue iteration k (0-based) with the index sets already on the device.
int enqueue_iter(ircur_ctx* c, int k, const int32_t* Id, const int32_t* Jd, const int32_t* Jhost) {
    const int slot = k % kRing;
    if (c->timing && c->acc_next <= k - kRing) {
        // the slot is about to be reused: its iteration has to be summed first
        for (int it = c->acc_next; it <= k - kRing; ++it) {
            HIPCHK(c, hipEventSynchronize(c->ev[it % kRing][4]));
            accumulate_timing(c, it);
        }
        c->acc_next = k - kRing + 1;
    }
    const ircur_params& p = c->p;
    const int cur = k & 1, nxt = cur ^ 1;
    const double zeta = zeta_at(c, k);
    const float zf = round_down_float(zeta);
    hipStream_t s = c->stream;
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[slot][0], s));

    bool sameJ = c->have_prevV && (int)c->lastJ.size() == p.sJ &&
                 std::equal(c->lastJ.begin(), c->lastJ.end(), Jhost);
    if (c->csvd) {
        CoreArgs ca{};
        ca.D = c->D; ca.ldD = p.ldD; ca.I = Id; ca.J = Jd; ca.sI = p.sI; ca.sJ = p.sJ;
        ca.n1 = p.n1; ca.n2 = p.n2; ca.At = c->At[cur]; ca.B = c->B[cur];
        ca.zeta = zeta; ca.zeta_f = zf; ca.M = c->M; ca.MA = c->MA; ca.MB = nullptr; ca.st = c->st;
        ca.Abc = c->Abc; ca.Bsc = c->Bsc;
        HIPCHK(c, launch_core(ca, p.dtype, c->R, s));
        CsvdArgs ka{};
        ka.D = c->D; ka.ldD = p.ldD; ka.I = Id; ka.J = Jd; ka.sI = p.sI; ka.sJ = p.sJ;
        ka.r = p.r; ka.R = c->R; ka.n1 = p.n1; ka.n2 = p.n2;
        ka.At = c->At[cur]; ka.B = c->B[cur];
        ka.MA = c->MA; ka.Abc = c->Abc; ka.Bsc = c->Bsc;
        ka.G = c->Gc;
        ka.xs = c->Xs;
        ka.max_it = p.svd_max_it > 0 ? p.svd_max_it : 256;
        ka.tol = p.svd_tol > 0 ? p.svd_tol : (p.dtype == IRCUR_F64 ? 1e-13 : (p.dtype == IRCUR_F32 ? 1e-9 : 1e-7));
        ka.tol_e = (p.dtype == IRCUR_BF16 && !(p.svd_tol > 0)) ? 1e-2 : 0.0;
        ka.warm = k == 0 ? 0 : (sameJ ? 1 : 2);
        ka.salt = sm_mix(p.seed ^ (0xA24BAED4963EE407ull * (uint64_t)(k + 1)));
        ka.prevV = c->prevV; ka.Zp = c->Zp; ka.Gp = c->Gp; ka.Xr = c->Xr; ka.rp = c->rp;
        ka.W = c->W; ka.V = c->V; ka.sigma = c->sigma;
        // (the row form only for the vector pass; the matrix-core pass reads the tiles)
        ka.rowI = c->p16 ? nullptr : c->rowI; ka.rowJ = c->p16 ? nullptr : c->rowJ;
        ka.qs = row_stride(c->R, (int)c->fsz);
        ka.rowIt = c->rowIt; ka.rowJt = c->rowJt;
        ka.GmI = c->GmI; ka.GmJ = c->GmJ; ka.scaleJ = c->scaleJ; ka.TAd = c->TAd;
        ka.info = c->info + k; ka.st = c->st;
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[slot][1], s));
        HIPCHK(c, launch_csvd(ka, p.dtype, c->csvd_lds, s));
#ifdef IRCUR_PHASE_PROFILE
        // profile builds: the same launch again, straight after (same inputs,
        // same outputs for a warm start other than the previous basis), timed
        // into the second set of phase timers
        if (ka.warm != 1 && std::getenv("IRCUR_PROFILE_REPEAT")) {
            ka.prof_slot = 1;
            HIPCHK(c, launch_csvd(ka, p.dtype, c->csvd_lds, s));
        }
#endif
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[slot][2], s));
    } else {
    CoreArgs ca{};
    ca.D = c->D; ca.ldD = p.ldD; ca.I = Id; ca.J = Jd; ca.sI = p.sI; ca.sJ = p.sJ;
    ca.n1 = p.n1; ca.n2 = p.n2; ca.At = c->At[cur]; ca.B = c->B[cur];
    ca.zeta = zeta; ca.zeta_f = zf; ca.M = c->M; ca.MA = c->MA; ca.st = c->st;
    ca.MB = c->lds_svd ? nullptr : c->MB;
    ca.Abc = c->Abc; ca.Bsc = c->Bsc;
    HIPCHK(c, launch_core(ca, p.dtype, c->R, s));
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[slot][1], s));

    SvdArgs sa{};
    sa.MA = c->MA; sa.MB = c->MB; sa.sI = p.sI; sa.sJ = p.sJ; sa.r = p.r; sa.R = c->R; sa.p = c->psvd;
    sa.G = c->G; sa.bs = c->bs;
    sa.max_it = p.svd_max_it > 0 ? p.svd_max_it : 64;
    // default: well below the rounding of the stored D (bf16 keeps 8 bits)
    sa.tol = p.svd_tol > 0 ? p.svd_tol : (p.dtype == IRCUR_F64 ? 1e-13 : (p.dtype == IRCUR_F32 ? 1e-9 : 1e-7));
    // BF16 storage, default tolerance: the subspace follows the run's stopping
    // residual, max(1e-7, 1e-2 e_k) (an SVD a hundred times finer than the
    // iterate it updates; the last iterations get 1e-7)
    sa.tol_e = (p.dtype == IRCUR_BF16 && !(p.svd_tol > 0)) ? 1e-2 : 0.0;
    sa.warm = k == 0 ? 0 : (sameJ ? 1 : 2);
    sa.salt = sm_mix(p.seed ^ (0xA24BAED4963EE407ull * (uint64_t)(k + 1)));
    sa.prevV = c->prevV; sa.prevV_out = c->prevV;
    sa.I = Id; sa.J = Jd; sa.n1 = p.n1; sa.n2 = p.n2;
    sa.At = c->At[cur]; sa.B = c->B[cur];
    sa.Zp = c->Zp; sa.Gp = c->Gp;
    sa.W = c->W; sa.V = c->V; sa.sigma = c->sigma;
    sa.rowI = c->rowI; sa.rowJ = c->rowJ; sa.GmI = c->GmI; sa.GmJ = c->GmJ; sa.scaleJ = c->scaleJ;
    sa.TAd = c->TAd;
    sa.qs = row_stride(c->R, (int)c->fsz);
    sa.info = c->info + k; sa.st = c->st;
    sa.Abc = c->Abc; sa.Bsc = c->Bsc; sa.Zr = c->Zr; sa.rp = c->rp;
    if (c->lds_svd) {
        sa.warm = (sa.warm & 0xff) | ((p.dtype == IRCUR_F64 ? 0 : 1) << 8);
        HIPCHK(c, launch_svdl(sa, c->svd_lds, s));
    } else {
        HIPCHK(c, launch_svd(sa, p.dtype, c->svd_lds, s));
    }
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[slot][2], s));
    }
    c->have_prevV = true;
    c->lastJ.assign(Jhost, Jhost + p.sJ);

    PassArgs pa = pass_args(c, k, Id, Jd);
    if (c->csvd) { pa.gapT = c->TAd; pa.gapinfo = c->info + k; pa.gapR = c->R; }   // the SVD's gap estimate
    HIPCHK(c, launch_pass(pa, p.dtype, c->R, s));
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[slot][3], s));

    FinArgs fa{};
    fa.part_row = c->part_row; fa.nrow = c->nwg_row; fa.part_col = c->part_col; fa.ncol = c->nwg_col;
    fa.k = k; fa.max_iter = p.max_iter; fa.eps = p.eps; fa.hist = c->hist; fa.st = c->st;
    HIPCHK(c, launch_finalize(fa, s));
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[slot][4], s));
    c->last_k = k;
    c->lastIdev = Id;
    c->lastJdev = Jd;
    return IRCUR_OK;
}

void sorted_copy(const int32_t* src, int32_t n, int32_t* dst) {
    std::copy(src, src + n, dst);
    std::sort(dst, dst + n);
}

// Enqueue iterations k0 .. k0+n-1 (k0 = next to enqueue) with sampled sets,
// or one iteration with the given pair.  Batches alternate between the two
// halves of the index-set ring; a half is rewritten only after the copy that
// last read its pinned host buffer has completed.
int enqueue_chunk(ircur_ctx* c, int n, const int32_t* Igiven, const int32_t* Jgiven) {
    const ircur_params& p = c->p;
    const int k0 = c->k_enq;
    if (n > kChunk) n = kChunk;
    const int h = c->batch & 1;
    if (c->h2d_pending[h]) {
        HIPCHK(c, hipEventSynchronize(c->h2d[h]));
        c->h2d_pending[h] = false;
    }
    // slot j of the batch: I (sI entries and the padding), then J
    const size_t strI = (size_t)p.sI + kIndexPad, strJ = (size_t)p.sJ + kIndexPad, strIJ = strI + strJ;
    int32_t* hbase = c->IJpin + (size_t)h * kChunk * strIJ;
    int32_t* dbase = c->IJdev + (size_t)h * kChunk * strIJ;
    for (int j = 0; j < n; ++j) {
        const int k = k0 + j;
        int32_t* Ih = hbase + (size_t)j * strIJ;
        int32_t* Jh = Ih + strI;
        if (Igiven) {
            sorted_copy(Igiven, p.sI, Ih);
            sorted_copy(Jgiven, p.sJ, Jh);
        } else {
            SplitMix64 g = index_stream(p.seed, p.resample ? k : 0);
            floyd(g, p.n1, p.sI, Ih);
            floyd(g, p.n2, p.sJ, Jh);
        }
        std::fill(Ih + p.sI, Ih + strI, Ih[p.sI - 1]);
        std::fill(Jh + p.sJ, Jh + strJ, Jh[p.sJ - 1]);
        if (k < p.max_iter) {
            std::copy(Ih, Ih + p.sI, c->setsI.begin() + (size_t)k * p.sI);
            std::copy(Jh, Jh + p.sJ, c->setsJ.begin() + (size_t)k * p.sJ);
        }
    }
    HIPCHK(c, hipMemcpyAsync(dbase, hbase, sizeof(int32_t) * n * strIJ, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipEventRecord(c->h2d[h], c->stream));
    c->h2d_pending[h] = true;
    c->batch += 1;
    for (int j = 0; j < n; ++j) {
        const int32_t* Id = dbase + (size_t)j * strIJ;
        const int rc = enqueue_iter(c, k0 + j, Id, Id + strI, hbase + (size_t)j * strIJ + strI);
        if (rc) return rc;
        c->k_enq = k0 + j + 1;
    }
    return IRCUR_OK;
}

}  // namespace

// ================================================================ C ABI ===

extern "C" {

int ircur_params_default(ircur_params* p) {
    if (!p) return IRCUR_ERR_ARG;
    std::memset(p, 0, sizeof(*p));
    p->gamma = 0.7;
    p->eps = 1e-5;
    p->max_iter = 100;
    p->resample = 1;
    p->err_mode = 0;
    p->dtype = IRCUR_F64;
    return IRCUR_OK;
}

int ircur_sample(uint64_t seed, int64_t t, int64_t n1, int64_t n2, int32_t sI, int32_t sJ,
                 int32_t* I_host, int32_t* J_host) {
    if (!I_host || !J_host || n1 < 1 || n2 < 1 || sI < 0 || sJ < 0 || sI > n1 || sJ > n2 || t < 0)
        return IRCUR_ERR_ARG;
    SplitMix64 g = index_stream(seed, t);
    floyd(g, n1, sI, I_host);
    floyd(g, n2, sJ, J_host);
    return IRCUR_OK;
}

int ircur_init(ircur_ctx** out, const ircur_params* pin, const void* D_dev, const void* Dt_dev,
               int64_t ldDt, void* stream) {
    if (!out) return IRCUR_ERR_ARG;
    *out = nullptr;
    int rc = validate(pin, D_dev, Dt_dev, ldDt);
    if (rc) return rc;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return IRCUR_ERR_DEVICE;

    ircur_ctx* c = new (std::nothrow) ircur_ctx();
    if (!c) return IRCUR_ERR_ALLOC;
    c->p = *pin;
    if (pin->zeta_sched) c->zsched.assign(pin->zeta_sched, pin->zeta_sched + pin->max_iter);
    c->p.zeta_sched = nullptr;               // (the copy above is the context's)
    const ircur_params& p = c->p;
    c->R = pad_rank(p.r);
    // SVD: tile width P = 16 or 32, the smaller one at least max(R, svd_block);
    // workgroups G the fewest of 8, 16, 32 whose LDS layout (M row block,
    // subspace blocks) fits in 160 KiB.
    const int P = std::max(c->R, (int)p.svd_block) <= 16 ? 16 : 32;
    int pb = P;
    size_t lds = 0;
    {
        // P = 16: the variant with the row block of M in LDS (fewest workgroups
        // of 8, 16, 32 that fit); otherwise, or if none fits, the streaming one.
        bool ok = false;
        if (P == 16) {
            for (int g : {8, 16, 32}) {
                const int bs = 16 * ((p.sI + 16 * g - 1) / (16 * g));
                const size_t l = svdl_lds_bytes(p.sJ, bs, g);
                if (l <= 160 * 1024) { c->G = g; c->bs = bs; lds = l; ok = true; c->lds_svd = true; break; }
            }
        }
        for (int g : {8, 16, 32}) {
            if (ok) break;
            c->G = g;
            c->bs = 16 * ((p.sI + 16 * g - 1) / (16 * g));   // rows per workgroup, multiple of 16
            lds = svd_lds_bytes(p.sJ, c->bs, P);
            if (lds <= 160 * 1024) { ok = true; break; }
        }
        if (!ok) { delete c; return IRCUR_ERR_UNSUPPORTED; }
    }
    c->psvd = pb;
    c->svd_lds = lds;
    {
        // one launch for the core and the SVD: R <= 16, one workgroup per 16
        // rows of M, all co-resident (at most one per compute unit), LDS fit
        int ncu = 0;
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 0;
        const int gc = (p.sI + 15) / 16;
        // (16 columns: a width above 16 takes the general SVD)
        if (P == 16 && gc <= ncu && p.sJ <= 512 && csvd_lds_bytes(p.sJ, gc) <= 160 * 1024) {
            c->csvd = true;
            c->Gc = gc;
            c->csvd_lds = csvd_lds_bytes(p.sJ, gc);
            // workgroups are dispatched to the XCDs in turn: a stride of the XCD
            // count puts the G working ones on one XCD (one per compute unit),
            // so their exchanges and barriers stay in that XCD's L2
            int nx = 1;
            if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || nx < 1) nx = 1;
            c->Xs = (nx > 1 && gc * nx <= ncu) ? nx : 1;
#ifdef IRCUR_PHASE_PROFILE
            if (std::getenv("IRCUR_SPREAD")) c->Xs = 1;
#endif
        }
    }
    c->stream = (hipStream_t)stream;
    (void)hipGetDevice(&c->device);
    if (!noalloc_setup(c->device)) { delete c; return IRCUR_ERR_DEVICE; }
    c->esz = p.dtype == IRCUR_F64 ? 8 : (p.dtype == IRCUR_F32 ? 4 : 2);
    c->fsz = p.dtype == IRCUR_F64 ? 8 : 4;
    c->D = D_dev;
    c->p16 = c->csvd && pass16_ok(p.dtype, c->R, std::max(p.sI, p.sJ));
    {
        const int pc = pass_cols(p.dtype, c->R, c->p16);
        c->nwg_row = (int)((p.n2 + pc - 1) / pc);
        c->nwg_col = (int)((p.n1 + pc - 1) / pc);
    }

#define TRY(x)                      \
    do {                            \
        int r_ = (x);               \
        if (r_) {                   \
            free_all(c);            \
            delete c;               \
            return r_;              \
        }                           \
    } while (0)
    const size_t R = c->R;
    for (int i = 0; i < 2; ++i) {
        TRY(dalloc_bytes(c, &c->At[i], R * p.n1 * c->fsz));
        TRY(dalloc_bytes(c, &c->B[i], R * p.n2 * c->fsz));
    }
    TRY(dalloc(c, &c->IJdev, (size_t)kRing * (p.sI + p.sJ + 2 * kIndexPad)));
    if (hipEventCreateWithFlags(&c->h2d[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->h2d[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->snap_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->snap_ev[1], hipEventDisableTiming) != hipSuccess) {
        free_all(c);
        delete c;
        return IRCUR_ERR_DEVICE;
    }
    if (hipHostMalloc((void**)&c->IJpin, sizeof(int32_t) * kRing * (p.sI + p.sJ + 2 * kIndexPad),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->st_host, sizeof(DevState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->snap_host, 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        free_all(c);
        delete c;
        return IRCUR_ERR_ALLOC;
    }
    TRY(dalloc(c, &c->M, (size_t)p.sI * p.sJ));
    {
        const size_t sI16 = ((size_t)p.sI + 15) / 16 * 16, sJ16 = ((size_t)p.sJ + 15) / 16 * 16;
        TRY(dalloc(c, &c->MA, sI16 * sJ16));
        TRY(dalloc(c, &c->MB, sI16 * sJ16));
        HIPCHK(c, hipMemset(c->MA, 0, sI16 * sJ16 * sizeof(double)));
        HIPCHK(c, hipMemset(c->MB, 0, sI16 * sJ16 * sizeof(double)));
    }
    {
        const size_t sI16 = ((size_t)p.sI + 15) / 16 * 16, sJ16 = ((size_t)p.sJ + 15) / 16 * 16;
        TRY(dalloc(c, &c->Zp, (size_t)c->G * sJ16 * c->psvd));
        if (c->lds_svd || c->csvd) {
            TRY(dalloc(c, &c->Abc, sI16 * 16));
            TRY(dalloc(c, &c->Bsc, 16 * sJ16));
            TRY(dalloc(c, &c->Zr, sJ16 * 16));
            TRY(dalloc(c, &c->rp, (size_t)c->G));
            HIPCHK(c, hipMemset(c->Abc, 0, sI16 * 16 * sizeof(double)));
            HIPCHK(c, hipMemset(c->Bsc, 0, 16 * sJ16 * sizeof(double)));
        }
    }
    TRY(dalloc(c, &c->Gp, (size_t)c->G * 2 * c->psvd * c->psvd));
    TRY(dalloc(c, &c->prevV, (size_t)p.sJ * R));
    if (c->csvd) {
        const size_t sJ16 = ((size_t)p.sJ + 15) / 16 * 16;
        // the one-launch SVD's partials, exchange block and basis of the last launch
        (void)hipFree(c->Zp); c->Zp = nullptr;
        (void)hipFree(c->Gp); c->Gp = nullptr;
        (void)hipFree(c->prevV); c->prevV = nullptr;
        TRY(dalloc(c, &c->Zp, (size_t)c->Gc * sJ16 * 16));
        TRY(dalloc(c, &c->Gp, (size_t)c->Gc * 768));
        TRY(dalloc(c, &c->prevV, sJ16 * 16));
        TRY(dalloc(c, &c->Xr, sJ16 * 16));
        if (!c->rp) TRY(dalloc(c, &c->rp, (size_t)c->Gc));
        else { (void)hipFree(c->rp); c->rp = nullptr; TRY(dalloc(c, &c->rp, (size_t)c->Gc)); }
        HIPCHK(c, hipMemset(c->Xr, 0, sJ16 * 16 * sizeof(double)));
    }
    TRY(dalloc(c, &c->W, (size_t)p.sI * R));
    TRY(dalloc(c, &c->V, (size_t)p.sJ * R));
    TRY(dalloc(c, &c->sigma, R * R));
    const size_t qs = (size_t)row_stride(c->R, (int)c->fsz);
    TRY(dalloc_bytes(c, &c->rowI, (size_t)p.sI * qs * c->fsz));
    TRY(dalloc_bytes(c, &c->rowJ, (size_t)p.sJ * qs * c->fsz));
    HIPCHK(c, hipMemset(c->rowI, 0, (size_t)p.sI * qs * c->fsz));
    HIPCHK(c, hipMemset(c->rowJ, 0, (size_t)p.sJ * qs * c->fsz));
    TRY(dalloc_bytes(c, &c->GmI, R * R * c->fsz));
    TRY(dalloc_bytes(c, &c->GmJ, R * R * c->fsz));
    TRY(dalloc_bytes(c, &c->scaleJ, R * R * c->fsz));
    TRY(dalloc(c, &c->TAd, R * R));
    TRY(dalloc(c, &c->Icur, (size_t)p.sI));
    TRY(dalloc(c, &c->Jcur, (size_t)p.sJ));
    TRY(dalloc(c, &c->nnz, 1));
    TRY(dalloc(c, &c->part_row, (size_t)2 * c->nwg_row));
    TRY(dalloc(c, &c->part_col, (size_t)2 * c->nwg_col));
    // (the matrix-core pass keeps every row of a column tile in one workgroup)
    c->ns_row = c->p16 ? 1 : pass_nsplit(p.dtype, c->R, p.sI, c->nwg_row);
    c->ns_col = c->p16 ? 1 : pass_nsplit(p.dtype, c->R, p.sJ, c->nwg_col);
    if (c->p16) {
        const size_t nbt = (size_t)(2 * ((c->R + 3) / 4) + 4) * 64 * c->fsz;
        TRY(dalloc_bytes(c, &c->rowIt, (size_t)((p.sI + 15) / 16) * nbt));
        TRY(dalloc_bytes(c, &c->rowJt, (size_t)((p.sJ + 15) / 16) * nbt));
    }
    {
        const size_t nblk = (size_t)c->nwg_row * c->ns_row + (size_t)c->nwg_col * c->ns_col;
        TRY(dalloc_bytes(c, &c->pacc, nblk * (pass_split_bytes(p.dtype, c->R) - 128 * sizeof(double))));
        TRY(dalloc(c, &c->pzd, nblk * 128));
        TRY(dalloc(c, &c->pcnt, (size_t)c->nwg_row + c->nwg_col));
        HIPCHK(c, hipMemset(c->pcnt, 0, sizeof(uint32_t) * ((size_t)c->nwg_row + c->nwg_col)));
    }
    TRY(dalloc(c, &c->st, 1));
    TRY(dalloc(c, &c->info, (size_t)p.max_iter));
    TRY(dalloc(c, &c->hist, (size_t)p.max_iter));
    c->setsI.assign((size_t)p.max_iter * p.sI, 0);
    c->setsJ.assign((size_t)p.max_iter * p.sJ, 0);
    if (Dt_dev) {
        c->Dt = Dt_dev;
        c->ldDt = ldDt;
    } else {
        // rows of D^T start on 128-byte boundaries (whole cache lines per column tile)
        const int64_t al = 128 / (int64_t)c->esz;
        c->ldDt = (p.n1 + al - 1) / al * al;
        TRY(dalloc_bytes(c, &c->Dt_own, (size_t)c->ldDt * p.n2 * c->esz));
        c->Dt = c->Dt_own;
        hipError_t e = launch_transpose(D_dev, p.ldD, c->Dt_own, c->ldDt, p.n1, p.n2, (int)c->esz, c->stream);
        if (e != hipSuccess) { free_all(c); delete c; return IRCUR_ERR_DEVICE; }
    }
    TRY(reset_state(c));
#undef TRY
    *out = c;
    return IRCUR_OK;
}

int ircur_reset(ircur_ctx* c) {
    if (!c) return IRCUR_ERR_ARG;
    return reset_state(c);
}

int ircur_step(ircur_ctx* c, const int32_t* I_host, const int32_t* J_host, double* e_out) {
    if (!c) return IRCUR_ERR_ARG;
    if ((I_host == nullptr) != (J_host == nullptr)) return fail(c, IRCUR_ERR_ARG, "give both I and J or neither");
    const ircur_params& p = c->p;
    if (I_host) {
        std::vector<int32_t> a(I_host, I_host + p.sI), b(J_host, J_host + p.sJ);
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        for (int i = 0; i < p.sI; ++i)
            if (a[i] < 0 || a[i] >= p.n1 || (i && a[i] == a[i - 1])) return fail(c, IRCUR_ERR_ARG, "I must hold distinct indices in [0, n1)");
        for (int i = 0; i < p.sJ; ++i)
            if (b[i] < 0 || b[i] >= p.n2 || (i && b[i] == b[i - 1])) return fail(c, IRCUR_ERR_ARG, "J must hold distinct indices in [0, n2)");
    }
    int rc = read_state(c);
    if (rc) return rc;
    if (c->stopped || c->k >= p.max_iter) return fail(c, IRCUR_ERR_STATE, "run already stopped");
    rc = enqueue_chunk(c, 1, I_host, J_host);
    if (rc) return rc;
    rc = read_state(c);
    if (rc) return rc;
    if (e_out) *e_out = c->st_host->e_last;
    return status_after(c);
}

int ircur_enqueue(ircur_ctx* c, int32_t n_iter) {
    if (!c || n_iter < 0) return IRCUR_ERR_ARG;
    while (n_iter > 0) {
        if (c->stopped || c->k_enq >= c->p.max_iter) break;
        const int n = std::min<int>(std::min(n_iter, kChunk), c->p.max_iter - c->k_enq);
        int rc = enqueue_chunk(c, n, nullptr, nullptr);
        if (rc) return rc;
        n_iter -= n;
    }
    return IRCUR_OK;
}

int ircur_sync(ircur_ctx* c, int32_t* k_out, double* e_out) {
    if (!c) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    if (k_out) *k_out = c->k;
    if (e_out) *e_out = c->st_host->e_last;
    return status_after(c);
}

int ircur_solve(ircur_ctx* c, int32_t* iters_out, double* e_out) {
    if (!c) return IRCUR_ERR_ARG;
    const ircur_params& p = c->p;
    int rc0 = read_state(c);
    if (rc0) return rc0;
    // Two chunks in flight: the next chunk is sampled and enqueued while the
    // device runs the current one, and the host waits only for a copy of the
    // device state taken after the older chunk.  Iterations enqueued past the
    // device-side stop return at once; chunks stay small (up to kSolveChunk)
    // so that few are enqueued past the stop.
    constexpr int kSolveChunk = 8;
    int chunk = 2;
    int inflight = 0, oldest = 0;
    bool seen_stop = c->stopped;
    while (true) {
        while (inflight < 2 && !seen_stop && c->k_enq < p.max_iter) {
            const int n = std::min(chunk, p.max_iter - c->k_enq);
            int rc = enqueue_chunk(c, n, nullptr, nullptr);
            if (rc) return rc;
            const int slot = (oldest + inflight) & 1;
            HIPCHK(c, hipMemcpyAsync(c->snap_host + slot, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipEventRecord(c->snap_ev[slot], c->stream));
            ++inflight;
            chunk = std::min(chunk * 2, kSolveChunk);
        }
        if (inflight == 0) break;
        HIPCHK(c, hipEventSynchronize(c->snap_ev[oldest]));
        const DevState& sn = c->snap_host[oldest];
        oldest ^= 1;
        --inflight;
        if (sn.stop || sn.svd_fail || sn.nonfinite || sn.k_done >= p.max_iter) seen_stop = true;
        if (seen_stop) break;
    }
    int rc = read_state(c);   // waits for the chunk still in flight (no-ops past the stop)
    if (rc) return rc;
    rc = status_after(c);
    if (rc) return rc;
    if (iters_out) *iters_out = c->k;
    const double e = c->k > 0 ? c->st_host->e_last : 1.0;
    if (e_out) *e_out = e;
    return (e <= p.eps) ? IRCUR_OK : IRCUR_NOT_CONVERGED;
}

int ircur_get_factors(ircur_ctx* c, void* At_dev, void* B_dev) {
    if (!c) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    const int cur = c->k & 1;
    const size_t r = c->p.r;
    if (At_dev) HIPCHK(c, hipMemcpyAsync(At_dev, c->At[cur], r * c->p.n1 * c->fsz, hipMemcpyDeviceToDevice, c->stream));
    if (B_dev) HIPCHK(c, hipMemcpyAsync(B_dev, c->B[cur], r * c->p.n2 * c->fsz, hipMemcpyDeviceToDevice, c->stream));
    return IRCUR_OK;
}

int ircur_set_factors(ircur_ctx* c, const void* At_dev, const void* B_dev, int32_t k) {
    if (!c || !At_dev || !B_dev || k < 0 || k >= c->p.max_iter) return IRCUR_ERR_ARG;
    const int cur = k & 1;
    const size_t r = c->p.r, R = c->R;
    HIPCHK(c, hipMemsetAsync(c->At[cur], 0, R * c->p.n1 * c->fsz, c->stream));
    HIPCHK(c, hipMemsetAsync(c->B[cur], 0, R * c->p.n2 * c->fsz, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->At[cur], At_dev, r * c->p.n1 * c->fsz, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->B[cur], B_dev, r * c->p.n2 * c->fsz, hipMemcpyDeviceToDevice, c->stream));
    DevState h{};
    h.k_done = k;
    *c->st_host = h;
    HIPCHK(c, hipMemcpyAsync(c->st, c->st_host, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->k = k;
    c->k_enq = k;
    c->k_base = k;
    c->acc_next = k;
    c->stopped = false;
    c->have_prevV = false;
    c->last_k = -1;
    return IRCUR_OK;
}

int ircur_get_history(ircur_ctx* c, double* e_host, int32_t cap, int32_t* n_out) {
    if (!c || (!e_host && cap > 0) || cap < 0) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    const int n = std::min(cap, c->k);
    if (n > 0) {
        HIPCHK(c, hipMemcpyAsync(e_host, c->hist, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (n_out) *n_out = n;
    return IRCUR_OK;
}

int ircur_get_sets(ircur_ctx* c, int32_t* I_host, int32_t* J_host) {
    if (!c || !I_host || !J_host) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    if (c->k < 1) return fail(c, IRCUR_ERR_STATE, "no completed iteration");
    const size_t k = c->k - 1;
    std::copy(c->setsI.begin() + k * c->p.sI, c->setsI.begin() + (k + 1) * c->p.sI, I_host);
    std::copy(c->setsJ.begin() + k * c->p.sJ, c->setsJ.begin() + (k + 1) * c->p.sJ, J_host);
    return IRCUR_OK;
}

int ircur_get_core(ircur_ctx* c, double* M_dev, double* W_dev, double* sigma_dev, double* V_dev) {
    if (!c) return IRCUR_ERR_ARG;
    const ircur_params& p = c->p;
    const size_t R = c->R, r = p.r;
    if (M_dev) HIPCHK(c, hipMemcpyAsync(M_dev, c->M, sizeof(double) * p.sI * p.sJ, hipMemcpyDeviceToDevice, c->stream));
    if (W_dev) HIPCHK(c, hipMemcpy2DAsync(W_dev, r * sizeof(double), c->W, R * sizeof(double), r * sizeof(double), p.sI, hipMemcpyDeviceToDevice, c->stream));
    if (V_dev) HIPCHK(c, hipMemcpy2DAsync(V_dev, r * sizeof(double), c->V, R * sizeof(double), r * sizeof(double), p.sJ, hipMemcpyDeviceToDevice, c->stream));
    if (sigma_dev) HIPCHK(c, hipMemcpy2DAsync(sigma_dev, r * sizeof(double), c->sigma, R * sizeof(double), r * sizeof(double), r, hipMemcpyDeviceToDevice, c->stream));
    return IRCUR_OK;
}

int ircur_get_cur(ircur_ctx* c, void* C_dev, void* Upinv_dev, void* R_dev, void* SI_dev, void* SJ_dev) {
    if (!c) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    if (c->k <= c->k_base) return fail(c, IRCUR_ERR_STATE, "no iteration completed since the factors were set");
    const ircur_params& p = c->p;
    const int it = c->k - 1;                 // 0-based index of the last completed iteration
    const int prev = it & 1;                 // its input factors
    HIPCHK(c, hipMemcpyAsync(c->Icur, c->setsI.data() + (size_t)it * p.sI, sizeof(int32_t) * p.sI,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->Jcur, c->setsJ.data() + (size_t)it * p.sJ, sizeof(int32_t) * p.sJ,
                             hipMemcpyHostToDevice, c->stream));
    CurArgs a{};
    a.D = c->D; a.ldD = p.ldD; a.Dt = c->Dt; a.ldDt = c->ldDt;
    a.I = c->Icur; a.J = c->Jcur; a.sI = p.sI; a.sJ = p.sJ; a.n1 = p.n1; a.n2 = p.n2;
    a.At = c->At[prev]; a.B = c->B[prev];
    a.zeta = zeta_at(c, it); a.zeta_f = round_down_float(a.zeta);
    a.Rout = R_dev; a.SI = SI_dev; a.Cout = C_dev; a.SJ = SJ_dev;
    if (R_dev || SI_dev || C_dev || SJ_dev) HIPCHK(c, launch_cur(a, p.dtype, c->R, c->stream));
    if (Upinv_dev)
        HIPCHK(c, launch_upinv(c->V, c->TAd, c->W, p.sI, p.sJ, c->R, Upinv_dev, p.dtype == IRCUR_F64 ? 0 : 1,
                               c->stream));
    // the pageable index copies above must not outlive this call's host data
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IRCUR_OK;
}

// Algorithm 2 on the current factors with the workspace ws: the Gram
// partials (2 x nwg x R x R doubles, every entry rewritten by the launch),
// then T1 and Tf (2 x R x R each, rewritten as well).
static int to_svd_with(ircur_ctx* c, double* ws, double* W_dev, double* sigma_dev, double* V_dev) {
    const ircur_params& p = c->p;
    const int nwg = alg2_groups(p);
    const size_t R = c->R;
    Alg2Args a{};
    const int cur = c->k & 1;
    a.X[0] = c->At[cur]; a.X[1] = c->B[cur];
    a.n[0] = p.n1; a.n[1] = p.n2;
    a.r = p.r; a.R = c->R; a.fdt = p.dtype == IRCUR_F64 ? 0 : 1; a.nwg = nwg;
    a.parts = ws;
    a.T1 = ws + 2 * (size_t)nwg * R * R;
    a.Tf = a.T1 + 2 * R * R;
    a.sigma_out = sigma_dev;
    a.out[0] = W_dev; a.out[1] = V_dev;
    HIPCHK(c, launch_alg2(a, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IRCUR_OK;
}

int ircur_to_svd(ircur_ctx* c, double* W_dev, double* sigma_dev, double* V_dev) {
    if (!c) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    if (!c->alg2_buf) {
        const size_t R = c->R;
        TRY_ALLOC(c, dalloc(c, &c->alg2_buf, alg2_doubles(alg2_groups(c->p), R)));
    }
    return to_svd_with(c, c->alg2_buf, W_dev, sigma_dev, V_dev);
}

int ircur_to_svd_noalloc(ircur_ctx* c, double* W_dev, double* sigma_dev, double* V_dev) {
    if (!c) return IRCUR_ERR_ARG;
    double* ws = noalloc_scratch(c->device);
    if (!ws) return fail(c, IRCUR_ERR_STATE, "no-allocation workspace not set up on this device");
    const size_t need = alg2_doubles(alg2_groups(c->p), (size_t)c->R);
    if (need > kScratchDoubles)
        return fail(c, IRCUR_ERR_UNSUPPORTED, "Algorithm 2 workspace exceeds the fixed no-allocation array");
    int rc = read_state(c);
    if (rc) return rc;
    return to_svd_with(c, ws, W_dev, sigma_dev, V_dev);
}

static SparseArgs sparse_args(const ircur_ctx* c, double zeta, void* S_dev, int64_t ldS) {
    const ircur_params& p = c->p;
    const int cur = c->k & 1;
    SparseArgs a{};
    a.D = c->D; a.ldD = p.ldD; a.n1 = p.n1; a.n2 = p.n2;
    a.At = c->At[cur]; a.B = c->B[cur];
    a.zeta = zeta < 0.0 ? zeta_at(c, c->k) : zeta;
    a.zeta_f = round_down_float(a.zeta);
    a.S = S_dev; a.ldS = ldS;
    return a;
}

int ircur_sparse_full(ircur_ctx* c, double zeta, void* S_dev, int64_t ldS, int64_t* nnz_out) {
    if (!c || !S_dev || ldS < c->p.n2 || std::isnan(zeta)) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    const ircur_params& p = c->p;
    SparseArgs a = sparse_args(c, zeta, S_dev, ldS);
    a.nnz = nnz_out ? c->nnz : nullptr;
    if (nnz_out) HIPCHK(c, hipMemsetAsync(c->nnz, 0, sizeof(unsigned long long), c->stream));
    HIPCHK(c, launch_sparse_full(a, p.dtype, c->R, c->stream));
    if (nnz_out) {
        unsigned long long h = 0;
        HIPCHK(c, hipMemcpyAsync(&h, c->nnz, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *nnz_out = (int64_t)h;
    }
    return IRCUR_OK;
}

int ircur_get_info(ircur_ctx* c, int32_t* svd_iters, double* svd_resid, double* gap, int32_t* kept) {
    if (!c) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    if (c->k < 1) return fail(c, IRCUR_ERR_STATE, "no completed iteration");
    SvdInfo h{};
    HIPCHK(c, hipMemcpy(&h, c->info + (c->k - 1), sizeof(SvdInfo), hipMemcpyDeviceToHost));
    if (svd_iters) *svd_iters = h.iters;
    if (svd_resid) *svd_resid = h.resid;
    if (gap) *gap = h.gap;
    if (kept) *kept = h.kept;
    return IRCUR_OK;
}

int ircur_get_svd_history(ircur_ctx* c, int32_t* iters_host, double* gap_host, int32_t* kept_host,
                          int32_t cap, int32_t* n_out) {
    if (!c || cap < 0 || (cap > 0 && !iters_host && !gap_host && !kept_host)) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    const int first = c->k_base, n = std::min(cap, c->k - c->k_base);
    if (n > 0) {
        std::vector<SvdInfo> h((size_t)n);
        HIPCHK(c, hipMemcpyAsync(h.data(), c->info + first, sizeof(SvdInfo) * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int i = 0; i < n; ++i) {
            if (iters_host) iters_host[i] = h[i].iters;
            if (gap_host) gap_host[i] = h[i].gap;
            if (kept_host) kept_host[i] = h[i].kept;
        }
    }
    if (n_out) *n_out = n > 0 ? n : 0;
    return IRCUR_OK;
}

int ircur_set_timing(ircur_ctx* c, int32_t enable) {
    if (!c) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    c->acc_next = c->k;
    if (enable && !c->ev_made) {
        for (int i = 0; i < kRing; ++i)
            // timing-only events: no system-scope fence (no cache write-back
            // between the kernels that they bracket)
            for (int j = 0; j < 5; ++j)
                HIPCHK(c, hipEventCreateWithFlags(&c->ev[i][j], hipEventDisableSystemFence));
        c->ev_made = true;
    }
    c->timing = enable != 0;
    c->tsum[0] = c->tsum[1] = c->tsum[2] = c->tsum[3] = 0.0;
    c->tcount = 0;
    return IRCUR_OK;
}

int ircur_get_timing(ircur_ctx* c, double* ms4, int64_t* count) {
    if (!c || !ms4) return IRCUR_ERR_ARG;
    for (int q = 0; q < 4; ++q) ms4[q] = c->tsum[q];
    if (count) *count = c->tcount;
    return IRCUR_OK;
}

int ircur_time_pass(ircur_ctx* c, int32_t reps, double* us_out) {
    if (!c || reps < 1 || !us_out) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    if (c->k < 1 || c->stopped || c->last_k != c->k - 1)
        return fail(c, IRCUR_ERR_STATE, "time_pass needs a finished iteration of a run that has not stopped");
    // the pass of iteration k-1 reads A_{k-1}, B_{k-1} and the svd's per-row
    // data, all still in place, and rewrites A_k, B_k with the same values
    const PassArgs pa = pass_args(c, c->k - 1, c->lastIdev, c->lastJdev);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    if (he == hipSuccess) he = hipEventRecord(e0, c->stream);
    for (int i = 0; i < reps && he == hipSuccess; ++i) he = launch_pass(pa, c->p.dtype, c->R, c->stream);
    if (he == hipSuccess) he = hipEventRecord(e1, c->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (he != hipSuccess) return fail(c, IRCUR_ERR_DEVICE, hipGetErrorString(he));
    *us_out = 1e3 * (double)ms / reps;
    return IRCUR_OK;
}

int ircur_time_sparse(ircur_ctx* c, double zeta, void* S_dev, int64_t ldS, int32_t reps, double* us_out) {
    if (!c || !S_dev || ldS < c->p.n2 || std::isnan(zeta) || reps < 1 || !us_out) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    const SparseArgs a = sparse_args(c, zeta, S_dev, ldS);   // no count: nothing read back per launch
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    if (he == hipSuccess) he = hipEventRecord(e0, c->stream);
    for (int i = 0; i < reps && he == hipSuccess; ++i) he = launch_sparse_full(a, c->p.dtype, c->R, c->stream);
    if (he == hipSuccess) he = hipEventRecord(e1, c->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (he != hipSuccess) return fail(c, IRCUR_ERR_DEVICE, hipGetErrorString(he));
    *us_out = 1e3 * (double)ms / reps;
    return IRCUR_OK;
}

int ircur_get_state(ircur_ctx* c, void* buf, size_t* bytes) {
    if (!c || !bytes) return IRCUR_ERR_ARG;
    const ircur_params& p = c->p;
    const size_t fa = (size_t)c->R * p.n1 * c->fsz, fb = (size_t)c->R * p.n2 * c->fsz;
    const size_t need = 64 + fa + fb + sizeof(double) * p.max_iter;
    if (!buf) { *bytes = need; return IRCUR_OK; }
    if (*bytes < need) return fail(c, IRCUR_ERR_ARG, "state buffer too small");
    int rc = read_state(c);
    if (rc) return rc;
    char* o = (char*)buf;
    std::memset(o, 0, 64);
    const int64_t hdr[6] = {0x49524355520001LL, c->k, c->stopped ? 1 : 0, p.n1, p.n2, c->R};
    std::memcpy(o, hdr, sizeof(hdr));
    const int cur = c->k & 1;
    HIPCHK(c, hipMemcpy(o + 64, c->At[cur], fa, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(o + 64 + fa, c->B[cur], fb, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(o + 64 + fa + fb, c->hist, sizeof(double) * p.max_iter, hipMemcpyDeviceToHost));
    *bytes = need;
    return IRCUR_OK;
}

int ircur_set_state(ircur_ctx* c, const void* buf, size_t bytes) {
    if (!c || !buf) return IRCUR_ERR_ARG;
    const ircur_params& p = c->p;
    const size_t fa = (size_t)c->R * p.n1 * c->fsz, fb = (size_t)c->R * p.n2 * c->fsz;
    const size_t need = 64 + fa + fb + sizeof(double) * p.max_iter;
    if (bytes < need) return fail(c, IRCUR_ERR_ARG, "state buffer too small");
    int64_t hdr[6];
    std::memcpy(hdr, buf, sizeof(hdr));
    if (hdr[0] != 0x49524355520001LL || hdr[3] != p.n1 || hdr[4] != p.n2 || hdr[5] != c->R ||
        hdr[1] < 0 || hdr[1] > p.max_iter)
        return fail(c, IRCUR_ERR_ARG, "state does not match this context");
    const int k = (int)hdr[1];
    const char* o = (const char*)buf;
    const int cur = k & 1;
    HIPCHK(c, hipMemcpy(c->At[cur], o + 64, fa, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->B[cur], o + 64 + fa, fb, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->hist, o + 64 + fa + fb, sizeof(double) * p.max_iter, hipMemcpyHostToDevice));
    double e_last = 1.0;
    if (k > 0) std::memcpy(&e_last, o + 64 + fa + fb + sizeof(double) * (k - 1), sizeof(double));
    DevState h{};
    h.k_done = k;
    h.stop = (int32_t)hdr[2];
    h.e_last = e_last;
    HIPCHK(c, hipMemcpy(c->st, &h, sizeof(DevState), hipMemcpyHostToDevice));
    c->k = k;
    c->k_enq = k;
    c->k_base = k;
    c->acc_next = k;
    c->stopped = hdr[2] != 0;
    c->have_prevV = false;
    c->last_k = -1;
    return IRCUR_OK;
}

int ircur_get_phase_profile(ircur_ctx* c, double* us16) {
    if (!c || !us16) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    for (int i = 0; i < 16; ++i) us16[i] = (double)c->st_host->phase[i] * 0.01;   // 100 MHz ticks
    return IRCUR_OK;
}

int ircur_get_phase_profile2(ircur_ctx* c, double* us16) {
    if (!c || !us16) return IRCUR_ERR_ARG;
    int rc = read_state(c);
    if (rc) return rc;
    for (int i = 0; i < 16; ++i) us16[i] = (double)c->st_host->phase2[i] * 0.01;
    return IRCUR_OK;
}

void ircur_destroy(ircur_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

const char* ircur_strerror(int s) {
    switch (s) {
        case IRCUR_OK: return "ok";
        case IRCUR_NOT_CONVERGED: return "iteration cap reached before e <= eps";
        case IRCUR_WARN_RANK_DEFICIENT: return "components of U^+ dropped (rank-deficient core)";
        case IRCUR_WARN_SVD_INEXACT: return "top-r SVD reached its iteration cap";
        case IRCUR_ERR_ARG: return "invalid argument";
        case IRCUR_ERR_ALLOC: return "device allocation failed";
        case IRCUR_ERR_DEVICE: return "HIP error or no device";
        case IRCUR_ERR_SVD: return "SVD failure";
        case IRCUR_ERR_NONFINITE: return "non-finite value";
        case IRCUR_ERR_STATE: return "invalid state for this call";
        case IRCUR_ERR_UNSUPPORTED: return "sizes beyond a kernel limit";
        default: return "unknown status";
    }
}

const char* ircur_last_error(const ircur_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
