// Internal declarations shared by the IRCUR HIP kernels and the host runtime.
// Not part of the public ABI (see include/ircur.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ircur {

// Padded ranks the factor kernels are compiled for; a rank r runs as the
// smallest entry >= r with the extra factor rows held at zero.
constexpr int kRanks[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32};
// Trailing entries after every stored index set (copies of its last index):
// the pass kernel reads up to RowsInFlight - 1 (<= 63) indices past the rows
// a wave uses, so the padding must be at least the largest RowsInFlight.
constexpr int kIndexPad = 64;

// Row stride (elements) of the per-row data of the pass: 3R rounded up to a
// multiple of 16 bytes.
template <typename F, int R> struct RowStride {
    static constexpr int value = ((3 * R * (int)sizeof(F) + 15) / 16) * (16 / (int)sizeof(F));
};
inline int row_stride(int R, int fsz) { return ((3 * R * fsz + 15) / 16) * (16 / fsz); }
// Row split of the pass: rows per row block (about 128, so that each wave
// has a few groups of rows in flight) and the largest number of blocks per
// column tile.
constexpr int kPassSplitRows = 128;
constexpr int kPassMaxSplit = 64;
// Output columns of one pass column tile: 16 for the matrix-core pass
// (padded ranks up to kPass16MaxRank), 64 lanes x the columns per lane above.
constexpr int kPass16MaxRank = 16;
constexpr int kPass16MinRank = 8;
constexpr int kPass16MaxRows = 1024;
// The matrix-core pass applies: kPass16MinRank <= R <= kPass16MaxRank (below,
// the 16-row operand of the projection product is mostly padding and the
// vector pass moves fewer bytes), at most kPass16MaxRows sampled rows per side
// (their indices are staged in LDS), and the per-row data written in
// operand-tile order (by the one-launch SVD).
bool pass16_ok(int dtype, int R, int smax);
int pass_cols(int dtype, int R, bool matrix_core);
size_t pass16_lds_bytes(int dtype, int R, int s);

inline int pad_rank(int r) {
    for (int v : kRanks) if (v >= r) return v;
    return -1;
}

// Device-resident run state (one per context).  Written only by kernels,
// read by the host after a synchronisation.
struct DevState {
    int32_t stop;        // 1 once e <= eps, k = max_iter or an error occurred
    int32_t k_done;      // completed iterations
    int32_t nonfinite;   // a NaN/Inf was met
    int32_t svd_fail;    // the SVD's grid barrier timed out
    int32_t svd_capped;  // an SVD hit its iteration cap
    int32_t rank_drop;   // a component of U^+ was dropped by the pinv rule
    double e_last;
    uint32_t bar_ctr;    // grid-barrier counter of the SVD kernel
    uint32_t bar_exit;   // workgroups of the one-launch SVD past their last barrier
    uint64_t phase[16];  // phase timers (100 MHz ticks), only with IRCUR_PHASE_PROFILE
    uint64_t phase2[16]; // the same for a repeated launch (profile builds)
    int32_t prof_slot;   // which of the two the next launch accumulates into
    int32_t pad2_;
};

// Per-iteration SVD diagnostics, one record per iteration.
struct SvdInfo {
    int32_t iters;
    int32_t kept;
    double resid;        // max_i ||M^T w_i - sigma_i v_i|| / sigma_1
    double gap;          // sigma_{r+1} / sigma_r (Ritz estimate, 0 if p == r)
    double bx;           // one-launch SVD: the extra columns' largest Rayleigh quotient
                         // (~ sigma_{r+1}^2; -1 without extra columns), which a
                         // spare workgroup of the pass launch turns into gap
};

// Arguments of the fused row/column pass.  "Side" 0 is the row pass over
// D[I, :] (output B_{k+1}); side 1 is the column pass over D^T[J, :] (output
// A_{k+1}^T).  Both have the same shape: s gathered rows of length n.
struct SideArgs {
    const void* X;         // D (side 0) or D^T (side 1)
    int64_t ldX;
    const int32_t* rows;   // I or J, s entries
    int32_t s;
    int64_t n;             // row length (n2 or n1)
    const void* P;         // B_k (side 0) or A_k^T (side 1): R x n, row stride n
    const void* rowdata;   // s x QS (QS = row_stride): [gathered factor | projection | Delta]
    const void* tiled;     // the same in operand-tile order for the matrix-core pass
                           // (ceil(s/16) blocks of (2 ceil(R/4) + 4) x 64), or nullptr
    const void* Gm;        // R x R: Gamma (side 0) or Gamma'^T (side 1)
    const void* outmat;    // R x R map applied to the output row (nullptr: identity)
    void* out;             // new factor, R x n, row stride n
    double* part;          // 2 doubles per column tile: (residual, ||D_side||^2)
    int32_t nwg;           // column tiles (64 columns in the vector pass, 32 in the matrix-core one)
    // row split: nsplit workgroups per column tile, each over a block of
    // ceil(s / nsplit) rows; their partial sums meet in pacc/pzd and the last
    // workgroup of the tile to finish (ticket in cnt) adds them in block order
    // and writes the tile's output.  nsplit <= 1: one workgroup per tile.
    int32_t nsplit;
    void* pacc;            // nwg x nsplit x R x V x 64 (F)
    double* pzd;           // nwg x nsplit x 2 x 64
    uint32_t* cnt;         // nwg tickets, zero between launches
};

struct PassArgs {
    SideArgs side[2];
    double zeta;           // threshold zeta_{k+1}
    float zeta_f;          // largest float <= zeta (exact float comparison)
    int32_t err_mode;
    const DevState* st;
    // one-launch SVD (else nullptr): one more workgroup estimates the gap of
    // the iteration's SVD from gapinfo->bx and Ly^-T (gapR x gapR)
    const double* gapT;
    SvdInfo* gapinfo;
    int32_t gapR;
};

struct CoreArgs {
    const void* D; int64_t ldD;
    const int32_t* I; const int32_t* J;
    int32_t sI, sJ;
    int64_t n1, n2;
    const void* At;        // A_k^T, R x n1
    const void* B;         // B_k, R x n2
    double zeta; float zeta_f;
    double* M;             // sI x sJ, double, row-major
    // The same matrix in two layouts for the SVD's matrix-core products, each
    // made of 64-double blocks in lane order, zero outside sI x sJ:
    //   MA block (ti, ks), ti < sI16/16, ks < sJ16/4:  lane l holds
    //      M[16 ti + l%16][4 ks + l/16]            (A operand of M Q)
    //   MB block (tj, ks), tj < sJ16/16, ks < sI16/4:  lane l holds
    //      M[4 ks + l/16][16 tj + l%16]            (A operand of M^T Y)
    double* MA;
    double* MB;            // nullptr when the SVD does not read it
    // Compact copies of the sampled factor rows/columns for the SVD (doubles,
    // zero padded, nullptr if not needed): Abc[a * 16 + c] = A_k[I_a, c]
    // (sI16 x 16), Bsc[c * sJ16 + b] = B_k[c, J_b] (16 x sJ16).
    double* Abc;
    double* Bsc;
    DevState* st;
};

struct SvdArgs {
    const double* MA;      // M in the row-tiled layout (see CoreArgs)
    const double* MB;      // M in the column-tiled layout
    int32_t sI, sJ, r, R;
    int32_t p;             // tile width P (16 or 32) >= R
    int32_t G;             // workgroups
    int32_t bs;            // rows of M per workgroup (multiple of 16)
    int32_t max_it;
    double tol;
    double tol_e;          // > 0: the tolerance is max(tol, tol_e * e_k) (e_0 = 1)
    int32_t warm;          // 0 random, 1 previous right basis, 2 B_k[:, J]^T
    uint64_t salt;         // random fill salt
    const double* prevV;   // sJ x R (warm == 1)
    double* prevV_out;     // sJ x R
    const int32_t* I; const int32_t* J;
    int64_t n1, n2;
    const void* At;        // A_k^T (R x n1), factor dtype
    const void* B;         // B_k (R x n2), factor dtype
    double* Zp;            // G x sJ x P scratch
    double* Gp;            // G x 2 x P x P scratch
    double* W;             // sI x R out: orthonormal left basis Wt
    double* V;             // sJ x R out: orthonormal right basis Q
    double* sigma;         // R x R out: Kc with H_r(M) = Wt Kc Q^T
    void* rowI;            // sI x qs (factor dtype)
    void* rowJ;            // sJ x qs
    int32_t qs;            // row stride of rowI / rowJ (elements)
    void* GmI;             // R x R
    void* GmJ;             // R x R
    void* scaleJ;          // R x R: Ly^-T, the column side's output map
    double* TAd;           // R x R: Ly^-T in double (for U^+ on export)
    SvdInfo* info;         // one record (this iteration)
    DevState* st;
    // LDS-resident variant (P = 16): compact factor copies written by the
    // core kernel, the reduced Z (sJ16 x 16) and per-workgroup residual parts
    const double* Abc;     // sI16 x 16
    const double* Bsc;     // 16 x sJ16
    double* Zr;            // sJ16 x 16
    double* rp;            // G
};

// Core gather and top-r SVD in one launch (FP64 subspace arithmetic, R <= 16,
// G = ceil(sI / 16) workgroups, each owning 16 rows of M).
struct CsvdArgs {
    const void* D; int64_t ldD;
    const int32_t* I; const int32_t* J;
    int32_t sI, sJ, r, R;
    int64_t n1, n2;
    const void* At;        // A_k^T (R x n1), factor dtype
    const void* B;         // B_k (R x n2), factor dtype
    double zeta; float zeta_f;
    // the core [D - S_{k+1}]_{I,J} as written by the core kernel: row-tiled
    // layout (see CoreArgs::MA) and compact A_k[I, :] (sI16 x 16), B_k[:, J]
    // (16 x sJ16), zero padded
    const double* MA;
    const double* Abc;
    const double* Bsc;
    int32_t G;
    int32_t max_it;        // cap on applications of M^T M
    double tol;
    double tol_e;          // > 0: the tolerance is max(tol, tol_e * e_k) (e_0 = 1)
    int32_t warm;          // starting block: 0 random, 1 previous basis prevV, 2 B_k[:, J]^T
                           // (from Bsc) with pseudo-random extra columns
    uint64_t salt;         // pseudo-random entries of the starting block
    double* prevV;         // sJ16 x 16: basis of the previous launch (in for warm == 1; out)
    double* Zp;            // G x sJ16 x 16 partials
    double* Gp;            // G x 3 x 256 partials (Y^T Y, Y^T A_blk, B_k[:, J] Q)
    double* Xr;            // sJ16 x 16: the next block (exchange)
    double* rp;            // G residual parts
    double* W;             // sI x R out: orthonormal left basis Wt
    double* V;             // sJ x R out: orthonormal right basis Q
    double* sigma;         // R x R out: Kc with H_r(M) = Wt Kc Q^T
    void* rowI;            // sI x qs (factor dtype)
    void* rowJ;            // sJ x qs
    int32_t qs;
    void* rowIt;           // the per-row data in operand-tile order (see SideArgs::tiled), or nullptr
    void* rowJt;
    void* GmI; void* GmJ; void* scaleJ;
    double* TAd;
    SvdInfo* info;
    DevState* st;
    int32_t prof_slot;     // profile builds: phase timers of a repeated launch go to phase2
    int32_t xs;            // workgroup stride: the grid has G * xs workgroups and those with
                           // blockIdx % xs == 0 work (xs = number of XCDs: all on one XCD,
                           // whose L2 then holds the exchanged data; dispatch is round robin)
};

struct FinArgs {
    const double* part_row; int32_t nrow;
    const double* part_col; int32_t ncol;
    int32_t k;             // iteration index (0-based) being finished
    int32_t max_iter;
    double eps;
    double* hist;          // e history
    DevState* st;
};

// Export of the last completed iteration (C, R, S blocks), factor dtype out.
struct CurArgs {
    const void* D; int64_t ldD;
    const void* Dt; int64_t ldDt;
    const int32_t* I; const int32_t* J;
    int32_t sI, sJ;
    int64_t n1, n2;
    const void* At;        // A_{k-1}^T (input factors of that iteration)
    const void* B;         // B_{k-1}
    double zeta; float zeta_f;
    void* Rout;            // sI x n2 or nullptr
    void* SI;              // sI x n2 or nullptr
    void* Cout;            // n1 x sJ or nullptr
    void* SJ;              // n1 x sJ or nullptr
};

// Full sparse part T_zeta(D - A B), written in the dtype of D.
struct SparseArgs {
    const void* D; int64_t ldD;
    int64_t n1, n2;
    const void* At; const void* B;
    double zeta; float zeta_f;
    void* S; int64_t ldS;
    unsigned long long* nnz;   // accumulated count (nullptr: not counted)
};

// Algorithm 2 on the factored estimate (FP64).
struct Alg2Args {
    const void* X[2];      // A^T (R x n1), B (R x n2), factor dtype
    int64_t n[2];
    int32_t r, R;
    int32_t fdt;           // 0: double factors, 1: float factors
    int32_t nwg;           // gram workgroups per side
    double* parts;         // 2 x nwg x R x R
    double* T1;            // 2 x R x R: first-pass maps L1^-T
    double* Tf;            // 2 x R x R: output maps
    double* sigma_out;     // r, or nullptr
    double* out[2];        // W (n1 x r), V (n2 x r), or nullptr
};

// ---- unrolled mode (a batch of independent instances) --------------------
// Grouped launches map blockIdx.x to (instance b, local block) through an
// offset table off[0..nb] (off[b] = first block of instance b).

// Loss of one instance: Grams of [A_K | W*] (n1 rows) and [B_K^T | V*] (n2 rows).
struct ULoss {
    const void* At; const void* B;        // A_K^T (R x n1), B_K (R x n2), factor dtype
    const void* Ws; const void* Vs;       // W* (n1 x r), V* (n2 x r), factor dtype
    int64_t n1, n2;
    int32_t r, R;
    int32_t nwgA, nwgB;                   // gram blocks per side
    double* gpart;                        // (nwgA + nwgB) x (2R)^2 partials
    double* gsum;                         // 2 x (2R)^2 reduced Grams
    double* loss;                         // 1 value
    void* Abar; void* Bbar;               // loss adjoints out (R x n1, R x n2)
};

// Reverse sweep of one step of one instance.
struct UBack {
    const void* D; int64_t ldD;
    const void* Dt; int64_t ldDt;
    int64_t n1, n2;
    int32_t sI, sJ, r, R;
    const int32_t* I; const int32_t* J;   // this step's sets
    const int32_t* posJ;                  // n2: index of column j in J, or -1
    const void* At; const void* B;        // A_k^T, B_k (tape)
    const void* Abar1; const void* Bbar1; // adjoints of A_{k+1}, B_{k+1}
    void* Abar0; void* Bbar0;             // adjoints of A_k, B_k (out)
    double* partI;                        // nwg_row x sI x R
    double* partJ;                        // nwg_col x sJ x R
    double* partz;                        // nwg_row + nwg_col
    int32_t nwg_row, nwg_col;
    // forward SVD outputs of this step (tape)
    const double* Wt;                     // sI x R  (orthonormal left basis)
    const double* Q;                      // sJ x R  (orthonormal right basis)
    const double* Kc;                     // R x R   (H_r(M) = Wt Kc Q^T)
    const double* TAd;                    // R x R   (Ly^-T: A_{k+1} = C Q Ly^-T)
    const double* M;                      // sI x sJ core
    // adjoint-of-the-core workspace and outputs
    double* Mperp;                        // sI16 x sJ16: M - W_r Sigma V_r^T, zero padded
    double* Wr; double* Vr;               // sI x R, sJ x R singular vectors (columns >= r zero)
    double* Tp;                           // sJ x R: Q Ly^-T
    double* X1; double* X2;               // sI x R, sJ x R: M_bar = X1 V_r^T + W_r X2^T with
    double* X1b; double* X2b;             // X1 = X1 + X1b, X2 = X2 + X2b (W side + V side)
    double* P1; double* P2;               // sI x R, sJ x R workspace
    double* dz;                           // this step's zeta gradient (one value)
    int32_t* flags;                       // bit 0: CG did not converge, bit 1: rank < r
    DevState* st;                         // the instance's run state (phase timers of profile builds)
};

// Launchers (return hipError_t of the launch).
hipError_t launch_transpose(const void* src, int64_t lds, void* dst, int64_t ldd,
                            int64_t rows, int64_t cols, int elem_bytes, hipStream_t s);
hipError_t launch_core(const CoreArgs& a, int dtype, int R, hipStream_t s);
hipError_t launch_svd(const SvdArgs& a, int dtype, size_t lds_bytes, hipStream_t s);
// Batch of nb cores, arr_dev[b] per core (device array); G in {1, 2, 4, 8}, P = 16.
hipError_t launch_svd_batch(const SvdArgs* arr_dev, int nb, int G, int P, size_t lds_bytes, hipStream_t s);
// LDS-resident variant (P = 16): one core (G in {8, 16, 32}) or a batch (G in {2, 4, 8}).
hipError_t launch_svdl(const SvdArgs& a, size_t lds_bytes, hipStream_t s);
hipError_t launch_svdl_batch(const SvdArgs* arr_dev, int nb, int G, size_t lds_bytes, hipStream_t s);
hipError_t launch_pass(const PassArgs& a, int dtype, int R, hipStream_t s);
hipError_t launch_pass16(const PassArgs& a, int dtype, int R, hipStream_t s);
// Row blocks per column tile for a pass side with s rows (1: no split), and
// the partial-sum bytes per (tile, block) that a split needs.
int pass_nsplit(int dtype, int R, int s, int tiles);
size_t pass_split_bytes(int dtype, int R);
hipError_t launch_finalize(const FinArgs& a, hipStream_t s);
// Core gather and top-r SVD in one launch; its LDS bytes.
hipError_t launch_csvd(const CsvdArgs& a, int dtype, size_t lds_bytes, hipStream_t s);
size_t csvd_lds_bytes(int sJ, int G);
hipError_t launch_set_bar(DevState* st, hipStream_t s);
size_t svd_lds_bytes(int sJ, int bs16, int P);
// LDS bytes of the variant that keeps its row block of M in LDS (P = 16).
size_t svdl_lds_bytes(int sJ, int bs16, int G);
hipError_t launch_cur(const CurArgs& a, int dtype, int R, hipStream_t s);
hipError_t launch_upinv(const double* V, const double* TA, const double* W, int sI, int sJ, int R,
                        void* out, int dtype, hipStream_t s);
hipError_t launch_sparse_full(const SparseArgs& a, int dtype, int R, hipStream_t s);
hipError_t launch_alg2(const Alg2Args& a, hipStream_t s);
// unrolled mode
hipError_t launch_ucore(const CoreArgs* arr, const int32_t* off, int nb, int total_blocks, const double* zk,
                        double tau_rel, int dtype, int R, hipStream_t s);
hipError_t launch_upass(const PassArgs* arr, const int32_t* off, int nb, int total_blocks,
                        const double* zeta_k, double tau_rel, int dtype, int R, hipStream_t s);
hipError_t launch_uloss(const ULoss* arr, const int32_t* off, int nb, int total_blocks, int dtype, hipStream_t s);
hipError_t launch_ulossadj(const ULoss* arr, const int32_t* off, int nb, int total_blocks, const double* dloss,
                           int dtype, hipStream_t s);
hipError_t launch_ubpass(int phase, const UBack* arr, const int32_t* off, int nb, int total_blocks, int max_s,
                         const double* zk, double tau_rel, int dtype, int R, hipStream_t s);
hipError_t launch_ubsmall(const UBack* arr, int nb, int max_s16, int cg_max_it, double cg_tol, hipStream_t s);
hipError_t launch_ubreduce(const UBack* arr, const int32_t* off, int nb, int total_blocks, int dtype, hipStream_t s);
size_t ubsmall_lds_bytes(int max_s16);
hipError_t launch_udzeta(const double* dz_inst, int nb, int K, double* dzeta, hipStream_t s);

}  // namespace ircur
