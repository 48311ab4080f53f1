// Host runtime of the unrolled, differentiable mode (see include/ircur.h):
// a batch of independent instances advanced K iterations with learnable
// thresholds, the loss of the final estimates, and the reverse sweep.
//
// Every stage is one grouped launch over the whole batch; the per-(step,
// instance) launch arguments are built once at creation and live in device
// memory, so a forward pass is 3K + 2 launches and a backward pass 4K + 2.
// The tape (A_k, B_k for k = 0..K, the core M and its factored SVD for
// every step) stays in HBM; the gathered rows and columns are recomputed in
// the reverse sweep.
#include "ircur_internal.h"
#include <cstdio>
#include "../../include/ircur.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace ircur;

namespace {

constexpr int kUMaxS = 176;     // largest |I|, |J| of the unrolled mode
constexpr int kUMaxRank = 16;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct UHost {
    ircur_instance in;
    void* arena = nullptr;
    void* Dt_own = nullptr;
    int nwg_row = 0, nwg_col = 0, nwgA = 0, nwgB = 0;
    // buffers (device, inside the arena)
    int32_t* I = nullptr;       // K x (sI + pad)
    int32_t* J = nullptr;       // K x (sJ + pad)
    int32_t* posJ = nullptr;    // K x n2
    void* At = nullptr;         // (K+1) x R x n1
    void* B = nullptr;          // (K+1) x R x n2
    double* M = nullptr;        // K x sI x sJ
    double* MA = nullptr;
    double* MB = nullptr;
    double* Zp = nullptr;
    double* Gp = nullptr;
    double* Abc = nullptr;      // compact A_k[I, :] (sI16 x 16)
    double* Bsc = nullptr;      // compact B_k[:, J] (16 x sJ16)
    double* Zr = nullptr;       // reduced Z of the SVD (sJ16 x 16)
    double* rp = nullptr;       // SVD residual parts (G)
    double* W = nullptr;        // K x sI x R
    double* V = nullptr;        // K x sJ x R
    double* Kc = nullptr;       // K x R x R
    double* TAd = nullptr;      // K x R x R
    void* rowI = nullptr;
    void* rowJ = nullptr;
    void* GmI = nullptr;
    void* GmJ = nullptr;
    void* scaleJ = nullptr;
    SvdInfo* info = nullptr;    // K
    double* epart = nullptr;
    double* gpart = nullptr;
    double* gsum = nullptr;
    void* Abar[2] = {nullptr, nullptr};
    void* Bbar[2] = {nullptr, nullptr};
    double* partI = nullptr;
    double* partJ = nullptr;
    double* partz = nullptr;
    double* Mperp = nullptr;
    double* Wr = nullptr;
    double* Vr = nullptr;
    double* Tp = nullptr;
    double* X1 = nullptr;
    double* X2 = nullptr;
    double* X1b = nullptr;
    double* X2b = nullptr;
    double* P1 = nullptr;
    double* P2 = nullptr;
    std::vector<int32_t> Ih, Jh;   // host copies of the sets
};

}  // namespace

struct ircur_unrolled {
    int nb = 0, K = 0, r = 0, R = 0, dtype = 0;
    double tau_rel = 0.0;
    size_t fsz = 8, esz = 8;
    hipStream_t stream = nullptr;
    int G = 1, max_s = 0, max_sI16 = 0, max_sJ16 = 0, max_bs16 = 0;
    size_t svd_lds = 0;
    std::vector<UHost> inst;
    void* common = nullptr;      // argument tables, offsets, small shared arrays
    CoreArgs* d_core = nullptr;
    SvdArgs* d_svd = nullptr;
    SvdArgs* d_svd_warm = nullptr;     // the same, warm-started from the previous forward's subspaces
    PassArgs* d_pass = nullptr;
    ULoss* d_loss = nullptr;
    UBack* d_back = nullptr;
    int32_t* off_core = nullptr;
    int32_t* off_pass = nullptr;
    int32_t* off_gram = nullptr;
    int32_t* off_ladj = nullptr;
    int32_t* off_bred = nullptr;
    int tot_core = 0, tot_pass = 0, tot_gram = 0, tot_ladj = 0, tot_bred = 0;
    DevState* st = nullptr;      // nb
    double* loss = nullptr;      // nb
    double* dz_inst = nullptr;   // K x nb
    int32_t* flags = nullptr;    // nb
    double* zeta = nullptr;      // K: thresholds of the last forward pass
    bool forward_done = false;
    std::string err;
};

namespace {

int ufail(ircur_unrolled* u, int code, const char* msg) {
    if (u) u->err = msg;
    return code;
}

#define UCHK(u, x)                                                            \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            (u)->err = std::string(#x) + ": " + hipGetErrorString(e_);         \
            return IRCUR_ERR_DEVICE;                                          \
        }                                                                     \
    } while (0)

void ufree(ircur_unrolled* u) {
    for (auto& h : u->inst) {
        if (h.arena) (void)hipFree(h.arena);
        if (h.Dt_own) (void)hipFree(h.Dt_own);
    }
    if (u->common) (void)hipFree(u->common);
}

// Bump allocator over one device allocation.
struct Carve {
    size_t off = 0;
    char* base = nullptr;
    template <typename T> T* take(size_t count) {
        T* p = base ? (T*)(base + off) : nullptr;
        off += align256(count * sizeof(T) + 1);
        return p;
    }
};

int validate_instance(const ircur_instance& in, int r) {
    if (!in.D || !in.Wstar || !in.Vstar) return IRCUR_ERR_ARG;
    if (in.n1 < 1 || in.n2 < 1 || in.n1 > INT32_MAX || in.n2 > INT32_MAX || in.ldD < in.n2) return IRCUR_ERR_ARG;
    if (in.sI < r || in.sJ < r || in.sI > in.n1 || in.sJ > in.n2) return IRCUR_ERR_ARG;
    if (in.Dt && in.ldDt < in.n1) return IRCUR_ERR_ARG;
    if (in.sI > kUMaxS || in.sJ > kUMaxS) return IRCUR_ERR_UNSUPPORTED;
    return IRCUR_OK;
}

}  // namespace

extern "C" {

int ircur_unrolled_create(ircur_unrolled** out, const ircur_instance* inst, int32_t nb, int32_t r, int32_t K,
                          int32_t dtype, double tau_rel, void* stream) {
    if (!out) return IRCUR_ERR_ARG;
    *out = nullptr;
    if (!inst || nb < 1 || K < 1 || r < 1 || r > kUMaxRank || (dtype != IRCUR_F64 && dtype != IRCUR_F32) ||
        !(tau_rel >= 0.0) || !std::isfinite(tau_rel))
        return IRCUR_ERR_ARG;
    for (int b = 0; b < nb; ++b) {
        const int rc = validate_instance(inst[b], r);
        if (rc) return rc;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return IRCUR_ERR_DEVICE;
    ircur_unrolled* u = new (std::nothrow) ircur_unrolled();
    if (!u) return IRCUR_ERR_ALLOC;
    u->nb = nb;
    u->K = K;
    u->r = r;
    u->R = pad_rank(r);
    u->dtype = dtype;
    u->tau_rel = tau_rel;
    u->fsz = dtype == IRCUR_F64 ? 8 : 4;
    u->esz = u->fsz;
    u->stream = (hipStream_t)stream;
    u->inst.resize(nb);
    const int R = u->R;
    for (int b = 0; b < nb; ++b) {
        const ircur_instance& in = inst[b];
        u->max_s = std::max(u->max_s, (int)std::max(in.sI, in.sJ));
        u->max_sI16 = std::max(u->max_sI16, (in.sI + 15) / 16 * 16);
        u->max_sJ16 = std::max(u->max_sJ16, (in.sJ + 15) / 16 * 16);
    }
    // SVD workgroups per core: the fewest of 2, 4, 8 whose LDS layout (row
    // block of M resident in LDS) fits; all workgroups of the batch are
    // co-resident (one per CU)
    {
        bool ok = false;
        for (int g : {2, 4, 8}) {
            const int bs16 = 16 * ((u->max_sI16 / 16 + g - 1) / g);
            const size_t lds = svdl_lds_bytes(u->max_sJ16, bs16, g);
            if (lds <= 160 * 1024) {
                u->G = g;
                u->max_bs16 = bs16;
                u->svd_lds = lds;
                ok = true;
                break;
            }
        }
        if (!ok || (size_t)u->G * nb > 256) { delete u; return IRCUR_ERR_UNSUPPORTED; }
    }
    if (ubsmall_lds_bytes(std::max(u->max_sI16, u->max_sJ16)) > 160 * 1024) { delete u; return IRCUR_ERR_UNSUPPORTED; }

#define UTRY(x)                                     \
    do {                                            \
        int r_ = (x);                               \
        if (r_) { ufree(u); delete u; return r_; }  \
    } while (0)
#define UHIP(x)                                                                   \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) { ufree(u); delete u; return IRCUR_ERR_DEVICE; }    \
    } while (0)

    const size_t fsz = u->fsz;
    const int qs = row_stride(R, (int)fsz);
    for (int b = 0; b < nb; ++b) {
        UHost& h = u->inst[b];
        h.in = inst[b];
        const ircur_instance& in = h.in;
        const int64_t n1 = in.n1, n2 = in.n2;
        const int sI = in.sI, sJ = in.sJ;
        const int sI16 = (sI + 15) / 16 * 16, sJ16 = (sJ + 15) / 16 * 16;
        h.nwg_row = (int)((n2 + 63) / 64);      // F64 / F32 storage: 64 columns per pass workgroup
        h.nwg_col = (int)((n1 + 63) / 64);
        h.nwgA = (int)std::min<int64_t>(64, (n1 + 127) / 128);
        h.nwgB = (int)std::min<int64_t>(64, (n2 + 127) / 128);
        const int G = u->G, P = 16;
        for (int pass = 0; pass < 2; ++pass) {
            Carve cv;
            cv.base = (char*)h.arena;
            h.I = cv.take<int32_t>((size_t)K * (sI + kIndexPad));
            h.J = cv.take<int32_t>((size_t)K * (sJ + kIndexPad));
            h.posJ = cv.take<int32_t>((size_t)K * n2);
            h.At = cv.take<char>((size_t)(K + 1) * R * n1 * fsz);
            h.B = cv.take<char>((size_t)(K + 1) * R * n2 * fsz);
            h.M = cv.take<double>((size_t)K * sI * sJ);
            h.MA = cv.take<double>((size_t)sI16 * sJ16);
            h.MB = cv.take<double>((size_t)sI16 * sJ16);
            h.Zp = cv.take<double>((size_t)G * sJ16 * P);
            h.Gp = cv.take<double>((size_t)G * 2 * P * P);
            h.Abc = cv.take<double>((size_t)sI16 * 16);
            h.Bsc = cv.take<double>((size_t)16 * sJ16);
            h.Zr = cv.take<double>((size_t)sJ16 * 16);
            h.rp = cv.take<double>((size_t)G);
            h.W = cv.take<double>((size_t)K * sI * R);
            h.V = cv.take<double>((size_t)K * sJ * R);
            h.Kc = cv.take<double>((size_t)K * R * R);
            h.TAd = cv.take<double>((size_t)K * R * R);
            h.rowI = cv.take<char>((size_t)sI * qs * fsz);
            h.rowJ = cv.take<char>((size_t)sJ * qs * fsz);
            h.GmI = cv.take<char>((size_t)R * R * fsz);
            h.GmJ = cv.take<char>((size_t)R * R * fsz);
            h.scaleJ = cv.take<char>((size_t)R * R * fsz);
            h.info = cv.take<SvdInfo>((size_t)K);
            h.epart = cv.take<double>((size_t)2 * (h.nwg_row + h.nwg_col));
            h.gpart = cv.take<double>((size_t)(h.nwgA + h.nwgB) * 4 * R * R);
            h.gsum = cv.take<double>((size_t)8 * R * R + 2);
            for (int q = 0; q < 2; ++q) {
                h.Abar[q] = cv.take<char>((size_t)R * n1 * fsz);
                h.Bbar[q] = cv.take<char>((size_t)R * n2 * fsz);
            }
            h.partI = cv.take<double>((size_t)h.nwg_row * sI * R);
            h.partJ = cv.take<double>((size_t)h.nwg_col * sJ * R);
            h.partz = cv.take<double>((size_t)(h.nwg_row + h.nwg_col));
            h.Mperp = cv.take<double>((size_t)sI16 * sJ16);
            h.Wr = cv.take<double>((size_t)sI * R);
            h.Vr = cv.take<double>((size_t)sJ * R);
            h.Tp = cv.take<double>((size_t)sJ * R);
            h.X1 = cv.take<double>((size_t)sI * R);
            h.X2 = cv.take<double>((size_t)sJ * R);
            h.X1b = cv.take<double>((size_t)sI * R);
            h.X2b = cv.take<double>((size_t)sJ * R);
            h.P1 = cv.take<double>((size_t)sI * R);
            h.P2 = cv.take<double>((size_t)sJ * R);
            if (pass == 0) {
                if (hipMalloc(&h.arena, cv.off) != hipSuccess) { h.arena = nullptr; ufree(u); delete u; return IRCUR_ERR_ALLOC; }
                UHIP(hipMemsetAsync(h.arena, 0, cv.off, u->stream));
            }
        }
        // D^T
        if (!in.Dt) {
            if (hipMalloc(&h.Dt_own, (size_t)n1 * n2 * u->esz) != hipSuccess) { h.Dt_own = nullptr; ufree(u); delete u; return IRCUR_ERR_ALLOC; }
            UHIP(launch_transpose(in.D, in.ldD, h.Dt_own, n1, n1, n2, (int)u->esz, u->stream));
            h.in.Dt = h.Dt_own;
            h.in.ldDt = n1;
        }
        // index sets of every step: sampler stream k of this instance's seed
        h.Ih.assign((size_t)K * (sI + kIndexPad), 0);
        h.Jh.assign((size_t)K * (sJ + kIndexPad), 0);
        std::vector<int32_t> pos((size_t)K * n2, -1);
        for (int k = 0; k < K; ++k) {
            int32_t* Ik = h.Ih.data() + (size_t)k * (sI + kIndexPad);
            int32_t* Jk = h.Jh.data() + (size_t)k * (sJ + kIndexPad);
            ircur_sample(in.seed, k, n1, n2, sI, sJ, Ik, Jk);
            std::fill(Ik + sI, Ik + sI + kIndexPad, Ik[sI - 1]);
            std::fill(Jk + sJ, Jk + sJ + kIndexPad, Jk[sJ - 1]);
            for (int q = 0; q < sJ; ++q) pos[(size_t)k * n2 + Jk[q]] = q;
        }
        UHIP(hipMemcpyAsync(h.I, h.Ih.data(), h.Ih.size() * sizeof(int32_t), hipMemcpyHostToDevice, u->stream));
        UHIP(hipMemcpyAsync(h.J, h.Jh.data(), h.Jh.size() * sizeof(int32_t), hipMemcpyHostToDevice, u->stream));
        UHIP(hipMemcpyAsync(h.posJ, pos.data(), pos.size() * sizeof(int32_t), hipMemcpyHostToDevice, u->stream));
        UHIP(hipStreamSynchronize(u->stream));   // the host vectors above are pageable
    }

    // argument tables and offsets
    std::vector<CoreArgs> core((size_t)K * nb);
    std::vector<SvdArgs> svd((size_t)K * nb);
    std::vector<PassArgs> pas((size_t)K * nb);
    std::vector<ULoss> los(nb);
    std::vector<UBack> back((size_t)K * nb);
    std::vector<int32_t> oc(nb + 1, 0), op(nb + 1, 0), og(nb + 1, 0), ol(nb + 1, 0), ob(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        const UHost& h = u->inst[b];
        oc[b + 1] = oc[b] + (int)(((int64_t)h.in.sI * h.in.sJ + 255) / 256);
        op[b + 1] = op[b] + h.nwg_row + h.nwg_col;
        og[b + 1] = og[b] + h.nwgA + h.nwgB;
        ol[b + 1] = ol[b] + (int)((h.in.n1 + 255) / 256) + (int)((h.in.n2 + 255) / 256);
        ob[b + 1] = ob[b] + (h.in.sI * R + 255) / 256 + (h.in.sJ * R + 255) / 256 + 1;
    }
    u->tot_core = oc[nb];
    u->tot_pass = op[nb];
    u->tot_gram = og[nb];
    u->tot_ladj = ol[nb];
    u->tot_bred = ob[nb];
    {
        Carve cv;
        for (int pass = 0; pass < 2; ++pass) {
            cv.off = 0;
            cv.base = (char*)u->common;
            u->d_core = cv.take<CoreArgs>(core.size());
            u->d_svd = cv.take<SvdArgs>(svd.size());
            u->d_svd_warm = cv.take<SvdArgs>(svd.size());
            u->d_pass = cv.take<PassArgs>(pas.size());
            u->d_loss = cv.take<ULoss>(los.size());
            u->d_back = cv.take<UBack>(back.size());
            u->off_core = cv.take<int32_t>(nb + 1);
            u->off_pass = cv.take<int32_t>(nb + 1);
            u->off_gram = cv.take<int32_t>(nb + 1);
            u->off_ladj = cv.take<int32_t>(nb + 1);
            u->off_bred = cv.take<int32_t>(nb + 1);
            u->st = cv.take<DevState>(nb);
            u->loss = cv.take<double>(nb);
            u->dz_inst = cv.take<double>((size_t)K * nb);
            u->flags = cv.take<int32_t>(nb);
            u->zeta = cv.take<double>(K);
            if (pass == 0) {
                if (hipMalloc(&u->common, cv.off) != hipSuccess) { u->common = nullptr; ufree(u); delete u; return IRCUR_ERR_ALLOC; }
                UHIP(hipMemsetAsync(u->common, 0, cv.off, u->stream));
            }
        }
    }
    const int fd = dtype == IRCUR_F64 ? 0 : 1;
    for (int k = 0; k < K; ++k) {
        for (int b = 0; b < nb; ++b) {
            const UHost& h = u->inst[b];
            const ircur_instance& in = h.in;
            const int sI = in.sI, sJ = in.sJ;
            const size_t e = (size_t)k * nb + b;
            const int32_t* Ik = h.I + (size_t)k * (sI + kIndexPad);
            const int32_t* Jk = h.J + (size_t)k * (sJ + kIndexPad);
            char* At_k = (char*)h.At + (size_t)k * R * in.n1 * fsz;
            char* At_k1 = (char*)h.At + (size_t)(k + 1) * R * in.n1 * fsz;
            char* B_k = (char*)h.B + (size_t)k * R * in.n2 * fsz;
            char* B_k1 = (char*)h.B + (size_t)(k + 1) * R * in.n2 * fsz;
            double* M_k = h.M + (size_t)k * sI * sJ;
            DevState* st = u->st + b;

            CoreArgs& ca = core[e];
            ca.D = in.D; ca.ldD = in.ldD; ca.I = Ik; ca.J = Jk; ca.sI = sI; ca.sJ = sJ;
            ca.n1 = in.n1; ca.n2 = in.n2; ca.At = At_k; ca.B = B_k;
            ca.M = M_k; ca.MA = h.MA; ca.MB = nullptr; ca.st = st;
            ca.Abc = h.Abc; ca.Bsc = h.Bsc;

            SvdArgs& sa = svd[e];
            sa.MA = h.MA; sa.MB = h.MB; sa.sI = sI; sa.sJ = sJ; sa.r = u->r; sa.R = R; sa.p = 16;
            sa.G = u->G; sa.bs = 16 * (((sI + 15) / 16 + u->G - 1) / u->G);
            sa.max_it = 100;
            // FP32 data carry 24 significant bits: a subspace finer than about
            // their rounding (1e-7) buys nothing, and every extra order costs
            // ten power steps where sigma_{r+1} / sigma_r is near 0.9
            sa.tol = dtype == IRCUR_F64 ? 1e-13 : 1e-7;
            sa.warm = (k == 0 ? 0 : 2) | (fd << 8);
            sa.salt = in.seed * 0x9E3779B97F4A7C15ull + (uint64_t)(k + 1) * 0xD1B54A32D192ED03ull;
            sa.prevV = nullptr; sa.prevV_out = nullptr;
            sa.I = Ik; sa.J = Jk; sa.n1 = in.n1; sa.n2 = in.n2; sa.At = At_k; sa.B = B_k;
            sa.Zp = h.Zp; sa.Gp = h.Gp;
            sa.W = h.W + (size_t)k * sI * R; sa.V = h.V + (size_t)k * sJ * R;
            sa.sigma = h.Kc + (size_t)k * R * R;
            sa.rowI = h.rowI; sa.rowJ = h.rowJ; sa.qs = qs;
            sa.GmI = h.GmI; sa.GmJ = h.GmJ; sa.scaleJ = h.scaleJ;
            sa.TAd = h.TAd + (size_t)k * R * R;
            sa.info = h.info + k; sa.st = st;
            sa.Abc = h.Abc; sa.Bsc = h.Bsc; sa.Zr = h.Zr; sa.rp = h.rp;

            PassArgs& pa = pas[e];
            SideArgs& r0 = pa.side[0];
            r0.X = in.D; r0.ldX = in.ldD; r0.rows = Ik; r0.s = sI; r0.n = in.n2; r0.P = B_k;
            r0.rowdata = h.rowI; r0.Gm = h.GmI; r0.outmat = nullptr; r0.out = B_k1;
            r0.part = h.epart; r0.nwg = h.nwg_row;
            SideArgs& r1 = pa.side[1];
            r1.X = in.Dt; r1.ldX = in.ldDt; r1.rows = Jk; r1.s = sJ; r1.n = in.n1; r1.P = At_k;
            r1.rowdata = h.rowJ; r1.Gm = h.GmJ; r1.outmat = h.scaleJ; r1.out = At_k1;
            r1.part = h.epart + 2 * h.nwg_row; r1.nwg = h.nwg_col;
            pa.err_mode = 1; pa.st = st;

            UBack& ub = back[e];
            ub.D = in.D; ub.ldD = in.ldD; ub.Dt = in.Dt; ub.ldDt = in.ldDt; ub.n1 = in.n1; ub.n2 = in.n2;
            ub.sI = sI; ub.sJ = sJ; ub.r = u->r; ub.R = R;
            ub.I = Ik; ub.J = Jk; ub.posJ = h.posJ + (size_t)k * in.n2;
            ub.At = At_k; ub.B = B_k;
            ub.Abar1 = h.Abar[(k + 1) & 1]; ub.Bbar1 = h.Bbar[(k + 1) & 1];
            ub.Abar0 = h.Abar[k & 1]; ub.Bbar0 = h.Bbar[k & 1];
            ub.partI = h.partI; ub.partJ = h.partJ; ub.partz = h.partz;
            ub.nwg_row = h.nwg_row; ub.nwg_col = h.nwg_col;
            ub.Wt = sa.W; ub.Q = sa.V; ub.Kc = sa.sigma; ub.TAd = sa.TAd; ub.M = M_k;
            ub.Mperp = h.Mperp; ub.Wr = h.Wr; ub.Vr = h.Vr; ub.Tp = h.Tp; ub.X1 = h.X1; ub.X2 = h.X2; ub.X1b = h.X1b; ub.X2b = h.X2b;
            ub.P1 = h.P1; ub.P2 = h.P2;
            ub.dz = u->dz_inst + e;
            ub.flags = u->flags + b;
            ub.st = u->st + b;
        }
    }
    for (int b = 0; b < nb; ++b) {
        const UHost& h = u->inst[b];
        ULoss& L = los[b];
        L.At = (char*)h.At + (size_t)K * R * h.in.n1 * fsz;
        L.B = (char*)h.B + (size_t)K * R * h.in.n2 * fsz;
        L.Ws = h.in.Wstar; L.Vs = h.in.Vstar; L.n1 = h.in.n1; L.n2 = h.in.n2; L.r = u->r; L.R = R;
        L.nwgA = h.nwgA; L.nwgB = h.nwgB; L.gpart = h.gpart; L.gsum = h.gsum; L.loss = u->loss + b;
        L.Abar = h.Abar[K & 1]; L.Bbar = h.Bbar[K & 1];
    }
    UHIP(hipMemcpyAsync(u->d_core, core.data(), core.size() * sizeof(CoreArgs), hipMemcpyHostToDevice, u->stream));
    UHIP(hipMemcpyAsync(u->d_svd, svd.data(), svd.size() * sizeof(SvdArgs), hipMemcpyHostToDevice, u->stream));
    // later forward passes start each step's subspace iteration from the
    // subspace that the previous forward found for that step (its V_k, kept
    // in the tape and overwritten only by this step's own SVD, after every
    // workgroup has read it)
    std::vector<SvdArgs> svd_warm(svd);
    for (size_t e = 0; e < svd_warm.size(); ++e) {
        svd_warm[e].warm = 1 | (svd[e].warm & ~0xff);
        svd_warm[e].prevV = svd[e].V;
        svd_warm[e].prevV_out = nullptr;
    }
    UHIP(hipMemcpyAsync(u->d_svd_warm, svd_warm.data(), svd_warm.size() * sizeof(SvdArgs), hipMemcpyHostToDevice,
                        u->stream));
    UHIP(hipMemcpyAsync(u->d_pass, pas.data(), pas.size() * sizeof(PassArgs), hipMemcpyHostToDevice, u->stream));
    UHIP(hipMemcpyAsync(u->d_loss, los.data(), los.size() * sizeof(ULoss), hipMemcpyHostToDevice, u->stream));
    UHIP(hipMemcpyAsync(u->d_back, back.data(), back.size() * sizeof(UBack), hipMemcpyHostToDevice, u->stream));
    UHIP(hipMemcpyAsync(u->off_core, oc.data(), oc.size() * 4, hipMemcpyHostToDevice, u->stream));
    UHIP(hipMemcpyAsync(u->off_pass, op.data(), op.size() * 4, hipMemcpyHostToDevice, u->stream));
    UHIP(hipMemcpyAsync(u->off_gram, og.data(), og.size() * 4, hipMemcpyHostToDevice, u->stream));
    UHIP(hipMemcpyAsync(u->off_ladj, ol.data(), ol.size() * 4, hipMemcpyHostToDevice, u->stream));
    UHIP(hipMemcpyAsync(u->off_bred, ob.data(), ob.size() * 4, hipMemcpyHostToDevice, u->stream));
    UHIP(hipStreamSynchronize(u->stream));
#undef UTRY
#undef UHIP
    *out = u;
    return IRCUR_OK;
}

int ircur_unrolled_forward(ircur_unrolled* u, const double* zeta_dev, double* loss_dev) {
    if (!u || !zeta_dev) return IRCUR_ERR_ARG;
    const int nb = u->nb, R = u->R;
    UCHK(u, hipMemsetAsync(u->st, 0, sizeof(DevState) * nb, u->stream));
    UCHK(u, hipMemcpyAsync(u->zeta, zeta_dev, sizeof(double) * u->K, hipMemcpyDeviceToDevice, u->stream));
    for (int k = 0; k < u->K; ++k) {
        const size_t e = (size_t)k * nb;
        UCHK(u, launch_ucore(u->d_core + e, u->off_core, nb, u->tot_core, u->zeta + k, u->tau_rel, u->dtype, R,
                             u->stream));
        UCHK(u, launch_svdl_batch((u->forward_done ? u->d_svd_warm : u->d_svd) + e, nb, u->G, u->svd_lds,
                                  u->stream));
        UCHK(u, launch_upass(u->d_pass + e, u->off_pass, nb, u->tot_pass, u->zeta + k, u->tau_rel,
                             u->dtype, R, u->stream));
    }
    UCHK(u, launch_uloss(u->d_loss, u->off_gram, nb, u->tot_gram, u->dtype, u->stream));
    if (loss_dev)
        UCHK(u, hipMemcpyAsync(loss_dev, u->loss, sizeof(double) * nb, hipMemcpyDeviceToDevice, u->stream));
    u->forward_done = true;
    return IRCUR_OK;
}

int ircur_backward(ircur_unrolled* u, const double* dloss_dev, double* dzeta_dev) {
    if (!u || !dzeta_dev) return IRCUR_ERR_ARG;
    if (!u->forward_done) return ufail(u, IRCUR_ERR_STATE, "backward needs a forward pass first");
    const int nb = u->nb, R = u->R;
    UCHK(u, hipMemsetAsync(u->flags, 0, sizeof(int32_t) * nb, u->stream));
    UCHK(u, launch_ulossadj(u->d_loss, u->off_ladj, nb, u->tot_ladj, dloss_dev, u->dtype, u->stream));
    const int s16 = std::max(u->max_sI16, u->max_sJ16);
    // relative residual of the resolvent solves: far below the rounding of the
    // data and factors they serve (FP64: 1e-12; FP32: 1e-6)
    const double cg_tol = u->dtype == IRCUR_F64 ? 1e-12 : 1e-6;
    for (int k = u->K - 1; k >= 0; --k) {
        const UBack* arr = u->d_back + (size_t)k * nb;
        const double* zk = u->zeta + k;        // the forward pass's threshold of this step
        UCHK(u, launch_ubpass(1, arr, u->off_pass, nb, u->tot_pass, u->max_s, zk, u->tau_rel, u->dtype, R, u->stream));
        UCHK(u, launch_ubsmall(arr, nb, s16, 400, cg_tol, u->stream));
        UCHK(u, launch_ubpass(2, arr, u->off_pass, nb, u->tot_pass, u->max_s, zk, u->tau_rel, u->dtype, R, u->stream));
        UCHK(u, launch_ubreduce(arr, u->off_bred, nb, u->tot_bred, u->dtype, u->stream));
    }
    UCHK(u, launch_udzeta(u->dz_inst, nb, u->K, dzeta_dev, u->stream));
    return IRCUR_OK;
}

int ircur_unrolled_get_factors(ircur_unrolled* u, int32_t b, int32_t k, void* At_dev, void* B_dev) {
    if (!u || b < 0 || b >= u->nb || k < 0 || k > u->K) return IRCUR_ERR_ARG;
    const UHost& h = u->inst[b];
    const size_t fa = (size_t)u->r * h.in.n1 * u->fsz, fb = (size_t)u->r * h.in.n2 * u->fsz;
    const size_t sa = (size_t)u->R * h.in.n1 * u->fsz, sb = (size_t)u->R * h.in.n2 * u->fsz;
    if (At_dev) UCHK(u, hipMemcpyAsync(At_dev, (char*)h.At + k * sa, fa, hipMemcpyDeviceToDevice, u->stream));
    if (B_dev) UCHK(u, hipMemcpyAsync(B_dev, (char*)h.B + k * sb, fb, hipMemcpyDeviceToDevice, u->stream));
    return IRCUR_OK;
}

int ircur_unrolled_get_sets(ircur_unrolled* u, int32_t b, int32_t k, int32_t* I_host, int32_t* J_host) {
    if (!u || b < 0 || b >= u->nb || k < 0 || k >= u->K || !I_host || !J_host) return IRCUR_ERR_ARG;
    const UHost& h = u->inst[b];
    const int sI = h.in.sI, sJ = h.in.sJ;
    std::copy(h.Ih.begin() + (size_t)k * (sI + kIndexPad), h.Ih.begin() + (size_t)k * (sI + kIndexPad) + sI, I_host);
    std::copy(h.Jh.begin() + (size_t)k * (sJ + kIndexPad), h.Jh.begin() + (size_t)k * (sJ + kIndexPad) + sJ, J_host);
    return IRCUR_OK;
}

int ircur_unrolled_status(ircur_unrolled* u, int32_t* flags_host) {
    if (!u || !flags_host) return IRCUR_ERR_ARG;
    std::vector<int32_t> f(u->nb);
    std::vector<DevState> st(u->nb);
    UCHK(u, hipMemcpyAsync(f.data(), u->flags, sizeof(int32_t) * u->nb, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipMemcpyAsync(st.data(), u->st, sizeof(DevState) * u->nb, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
    int rc = IRCUR_OK;
    for (int b = 0; b < u->nb; ++b) {
        int32_t v = f[b];
        if (st[b].svd_capped) v |= 4;
        if (st[b].rank_drop) v |= 8;
        if (st[b].svd_fail) v |= 16;
        flags_host[b] = v;
        if (st[b].svd_fail) rc = IRCUR_ERR_SVD;
    }
    return rc;
}

void ircur_unrolled_destroy(ircur_unrolled* u) {
    if (!u) return;
    (void)hipStreamSynchronize(u->stream);
#ifdef IRCUR_PHASE_PROFILE
    {
        DevState h{};
        if (hipMemcpy(&h, u->st, sizeof(DevState), hipMemcpyDeviceToHost) == hipSuccess) {
            std::fprintf(stderr, "phases of instance 0 (total us; 0-8, 11: last forward's SVDs, 9-15: last backward's core adjoints):");
            for (int i = 0; i < 16; ++i) std::fprintf(stderr, " [%d] %.1f", i, (double)h.phase[i] * 0.01);
            std::fprintf(stderr, "\n");
        }
        // subspace iterations of the last forward's SVDs, per step (rows) and instance (columns)
        for (int k = 0; k < u->K; ++k) {
            std::fprintf(stderr, "svd iters k=%d:", k);
            for (size_t b = 0; b < u->inst.size(); ++b) {
                SvdInfo si{};
                if (hipMemcpy(&si, u->inst[b].info + k, sizeof(SvdInfo), hipMemcpyDeviceToHost) == hipSuccess)
                    std::fprintf(stderr, " %d", si.iters);
            }
            std::fprintf(stderr, "\n");
        }
    }
#endif
    ufree(u);
    delete u;
}

const char* ircur_unrolled_last_error(const ircur_unrolled* u) { return u ? u->err.c_str() : "null batch"; }

}  // extern "C"
