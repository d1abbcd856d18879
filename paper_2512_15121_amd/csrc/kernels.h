// Launch wrappers of the GIAMG device kernels (internal).
#pragma once

#include "internal.h"

namespace giamg {

// Hardware dispatches block b to XCD (b mod 8).  Logical block ids are
// reassigned so that each XCD receives one contiguous range of G blocks.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
    int64_t x = b & 7, i = b >> 3, q = G >> 3, r = G & 7;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Fused epilogues of the CSR product y_i = sum_j A_ij v_j, applied per row.
enum SpmvMode : int {
    SPMV_PLAIN = 0,      // y = A v
    SPMV_RESID = 1,      // y = f - A v
    SPMV_ADD = 2,        // y += A v                       (prolongation + correction)
    SPMV_CHEB_INIT = 3,  // r = dinv (f - A v), d_new = r / theta      (v = x)
    SPMV_CHEB_STEP = 4,  // r -= dinv A v, d_new = c1 v_i + c2 r, x update (v = d_old)
    SPMV_JACOBI = 5,     // y = v + omega dinv (f - A v)   (v = x_old, y = x_new)
    SPMV_DOT = 6,        // y = A v, block partials of v . y
    SPMV_DINV = 7,       // y = dinv A v
    SPMV_RINIT = 8,      // y = f - A v, block partials of f . f and y . y
    SPMV_RCHEB0 = 9,     // restriction fused with the next level's zero-start Chebyshev
                         // init: y = A v, r = dinv y, x = r / theta (x holds d_0)
};

// Row blocks of the streaming product: at most spmv_cap<T>() nonzeros (the
// LDS products) and spmv_threads<T>() rows per block of as many threads.
// FP64: 1024 threads, 8 nonzeros each; FP32: 512 threads, 16 each (the
// shapes measured fastest per precision).  Rows longer than the cap get a
// block each.
constexpr int SPMV_CAP = 8192;
constexpr int SPMV_CAP32 = 8192;
template <typename T>
constexpr int spmv_cap() { return sizeof(T) == 4 ? SPMV_CAP32 : SPMV_CAP; }
template <typename T>
constexpr int spmv_threads() { return sizeof(T) == 4 ? 512 : 1024; }
// The grouped form (opt-in) keeps blocks of 512 threads and 4096 entries.
constexpr int GROUP_THREADS = 512;
constexpr int GROUP_CAP = 4096;
// Lean form (small operators): threads per block; a block holds
// LEAN_THREADS / L rows.
constexpr int LEAN_THREADS = 256;

// flags of SPMV_CHEB_STEP
constexpr int CHEB_ASSIGN = 1;   // x = d_old (+ d_new) instead of x += ...
constexpr int CHEB_LAST = 2;     // add the new direction as well (last step)

// A row block of the CSR product form (DevCSR::bdesc): rows [r0, r0 + nrows)
// with n nonzeros from base; staged blocks own runs [run0, run0 + nruns).
// FP32 products of operators with at least this many nonzeros load the
// matrix stream with plain loads, smaller ones (and every FP64 product)
// non-temporal ones.  Measured on the MI355X (mixed solves, same bits
// either way): at 424 M nonzeros plain loads speed the FP32 products by
// ~3 % (solve 32.9 -> 33.9 solves/s); at 49 M they slow the solve by ~4 %
// (220 -> 210 solves/s: the stream then evicts what the rest of the
// V-cycle reuses from the caches); FP64 products lose ~2 % with them.
constexpr int64_t FP32_PLAIN_MIN_NNZ = int64_t(128) << 20;

struct BlockDesc {
    int64_t base, r0;
    int32_t nrows, n, run0, nruns;
};
static_assert(sizeof(BlockDesc) == 32, "BlockDesc layout");

// A block of the grouped product form (DevCSR::gblk, one more entry than
// blocks: block b spans entries [e0, next.e0), rows [r0, next.r0) of grows
// and groups [q0, next.q0) of ggrp; its g * E values start at v0).
struct GBlock {
    int64_t e0, v0;
    int32_t r0, q0, g, pad;
};
static_assert(sizeof(GBlock) == 32, "GBlock layout");

template <typename T>
struct SpmvArgs {
    const int64_t* rp = nullptr;
    const int32_t* ci = nullptr;
    const T* val = nullptr;
    int64_t n = 0;
    const T* v = nullptr;     // gathered vector
    T* y = nullptr;           // output (or d_new)
    const T* f = nullptr;
    const T* dinv = nullptr;
    T* r = nullptr;
    T* x = nullptr;
    double* partial = nullptr;
    T c1 = 0, c2 = 0, inv_theta = 0, omega = 0;
    int flags = 0;
    const int64_t* rblk = nullptr;   // row-block boundaries (nblk + 1 entries)
    const BlockDesc* bdesc = nullptr;  // per row block (nblk entries)
    int64_t nblk = 0;
    int block_cap = 0, block_threads = 0;   // shape the row blocks were built for
    int lanes = 16;                  // lanes that reduce one row (16, 4 or 1)
    const int* stop = nullptr;       // device stop flag (null: the thread's StopScope flag)
    const double* vnz = nullptr;     // SPMV_RINIT: when set and *vnz == 0, v is all +0 and
                                     // y = f exactly (A v = +0 row by row: every row has a
                                     // positive diagonal entry), so no product is formed
    // host only: events the dispatch itself records at kernel start and end
    // (timing; null for ordinary launches)
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    const int32_t* run_ptr = nullptr;   // staged gathers (DevCSR); null: every block gathers directly
    const int32_t* runs = nullptr;
    const uint16_t* slot = nullptr;
    int64_t nnz = 0, ncols = 0;      // host-side byte accounting only
    int64_t nnz_staged = 0, nruns = 0;
    // grouped form (DevCSR, build_grouping): when gblk is set the product
    // runs over nblk grouped blocks and reads gval / gslot / grows / ggrp
    // and the block run tables grun_ptr / gruns instead of the CSR arrays.
    const GBlock* gblk = nullptr;
    const int32_t* grows = nullptr;
    const uint32_t* ggrp = nullptr;   // per group: local entry offset << 16 | entries
    const uint16_t* gslot = nullptr;  // per entry: LDS slot of its column
    const int32_t* grun_ptr = nullptr;
    const int32_t* gruns = nullptr;
    const T* gval = nullptr;
    int64_t gentries = 0, ggroups = 0, gnruns = 0;   // host-side byte accounting only
    // lean form (DevCSR::lean): nblk blocks of LEAN_THREADS / lanes rows,
    // reading rp / ci / val / v directly
    bool lean = false;
};

template <typename T>
void launch_spmv(int mode, const SpmvArgs<T>& a, hipStream_t s);
// Median read bandwidth (GB/s) of a streaming kernel over `reps` reads of a
// fresh buffer of `bytes` bytes on the current device's null stream.
void read_bandwidth(int64_t bytes, int reps, double* gbs);
// Greedy row blocking of a CSR operator: consecutive rows while their
// nonzeros fit cap; the reduction width follows the mean row length.
void make_row_blocks(const int64_t* rp, int64_t n, int64_t cap, int64_t max_rows, std::vector<int64_t>& blocks,
                     int& lanes);
// Staged-gather tables of d (run_ptr, runs, slot) from its device CSR and
// row blocks; rp is the host copy of the row pointers.  Blocks whose columns
// span more than STAGE_SPAN or form more than b.threads runs, and
// long-row blocks, keep direct gathers.
constexpr int64_t STAGE_SPAN = 262144;
void build_staging(const DevCSR& d, RowBlocks& b, const std::vector<int64_t>& rp, hipStream_t s);
// Grouped form of d (groups.cpp): rows with identical column lists in groups
// of at most GROUP_ROWS, blocks of one group size, every block staged.  rp and
// ci are host copies of d's pattern.  Returns false (and leaves d without the
// form) when the form would not pay or an operator does not fit it.
constexpr int GROUP_ROWS = 8;
// Rows of a CSR pattern (host copy) with identical column lists: classes in
// order of their first row, rows ascending within a class.
std::vector<std::vector<int32_t>> identical_row_classes(const std::vector<int64_t>& rp,
                                                        const std::vector<int32_t>& ci, int64_t n);
bool build_grouping(DevCSR& d, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                    hipStream_t s);
// Values of the grouped form in FP32 (after make_fp32_values of the CSR).
void make_fp32_group_values(DevCSR& d, hipStream_t s);
// Device gather y[i] = x[idx[i]] (setup: value reordering).
void launch_gather_values(int64_t n, const int64_t* idx, const double* x, double* y, hipStream_t s);

// row-local kernels
template <typename T>
void launch_cheb_init0(int64_t n, const T* f, const T* dinv, T* r, T* d, T* x, T inv_theta,
                       bool write_x, hipStream_t s);
template <typename T>
void launch_jacobi0(int64_t n, const T* f, const T* dinv, T* x, T omega, hipStream_t s);
template <typename T>
void launch_copy(int64_t n, const T* a, T* b, hipStream_t s);
template <typename T>
void launch_add(int64_t n, const T* a, T* b, hipStream_t s);   // b += a
template <typename Tin, typename Tout>
void launch_convert(int64_t n, const Tin* a, Tout* b, hipStream_t s);
template <typename T>
void launch_coarse_apply(int64_t n, const double* inv, const T* f, T* x, hipStream_t s);
void launch_fill(int64_t n, double v, double* x, hipStream_t s);
// *flag = 1 if some x[i] has a nonzero bit pattern (flag must start at 0).
void launch_nonzero_flag(int64_t n, const double* x, double* flag, hipStream_t s);
// y = d .* x (elementwise; the diagonal preconditioner)
void launch_mul(int64_t n, const double* d, const double* x, double* y, hipStream_t s);

// reductions: block partials then a single-block finalize
int64_t vec_blocks(int64_t n);
// b: double, or float (widened exactly)
template <typename TB>
void launch_dot_partial(int64_t n, const double* a, const TB* b, double* partial, hipStream_t s);
template <typename TB>
void launch_dot2_partial(int64_t n, const double* a, const TB* b, const double* c,
                         double* partial, hipStream_t s);  // a.b and c.b
// CG scalar finalisations applied after a reduction (see ScalarSlot)
enum FinishKind : int {
    FIN_NONE = 0, FIN_ALPHA = 1, FIN_BETA_FIRST = 2, FIN_BETA = 3, FIN_BETA_FLEX = 4, FIN_CONV = 5
};
void launch_reduce(int64_t m, const double* partial, int64_t stride, int ncomp, double* out,
                   hipStream_t s, int fin = 0, double* scal = nullptr, int* ctl = nullptr);

// PCG / FCG vector kernels
// device scalar slots; (S_BB, S_RR) and (S_RZNEW, S_ZROLD) are written as pairs
enum ScalarSlot : int {
    S_BB = 0, S_RR = 1, S_RZ = 2, S_PQ = 3, S_ALPHA = 4, S_BETA = 5, S_RZNEW = 6, S_ZROLD = 7,
    S_FLAG = 8, S_TMP = 9, S_TOL = 10,
    S_XNZ = 11,   // 1 when the initial guess has a nonzero bit pattern, else 0
    S_COUNT = 16
};
// CG control block (device ints): stop flag, iterations done, iteration cap
enum CtlSlot : int { C_STOP = 0, C_ITERS = 1, C_MAXIT = 2, C_COUNT = 4 };

// While a StopScope is open, every kernel this thread launches through the
// wrappers of this header returns at once once *flag is nonzero.
class StopScope {
public:
    explicit StopScope(const int* flag);
    ~StopScope();
    StopScope(const StopScope&) = delete;
    StopScope& operator=(const StopScope&) = delete;
private:
    const int* prev_;
};
void launch_pcg_update(int64_t n, double* x, double* r, double* rold, const double* p,
                       const double* q, const double* scal, double* partial, hipStream_t s);
// The same update fused with the fine level's zero-start Chebyshev init of
// the next preconditioning: cr = dinv r_new, cd = cr inv_theta.
void launch_pcg_update_cheb0(int64_t n, double* x, double* r, const double* p, const double* q,
                             const double* scal, double* partial, const double* dinv, double* cr,
                             double* cd, double inv_theta, hipStream_t s);
// The flexible-CG update (r_old = r) that also writes r_new in FP32 to f32
// and, with dinv32 non-null, the fine level's FP32 Chebyshev init (cr, cd).
void launch_pcg_update_mixed(int64_t n, double* x, double* r, double* rold, const double* p,
                             const double* q, const double* scal, double* partial, float* f32,
                             const float* dinv32, float* cr, float* cd, float inv_theta, hipStream_t s);
// p = z + beta p; z double, or float (widened exactly)
template <typename TZ>
void launch_pcg_direction(int64_t n, const TZ* z, double* p, const double* scal, hipStream_t s);
void launch_power_start(int64_t n, double* v, hipStream_t s);
void launch_scale(int64_t n, double a, const double* x, double* y, hipStream_t s);

// blocked (multi right-hand side) kernels, row-major [n][k]
template <typename T>
void launch_spmm(int mode, const SpmvArgs<T>& a, int k, hipStream_t s);

}  // namespace giamg
