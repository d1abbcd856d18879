// Internal declarations of the GIAMG library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/giamg.h"

namespace giamg {

// ---- error handling -------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define GIAMG_HIP(call)                                                        \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            throw ::giamg::Error(GIAMG_EHIP, std::string(#call) + ": " +       \
                                                 hipGetErrorString(e_));       \
    } while (0)

#define GIAMG_REQUIRE(cond, msg)                                               \
    do {                                                                       \
        if (!(cond)) throw ::giamg::Error(GIAMG_EINVAL, msg);                  \
    } while (0)

// ---- device memory ----------------------------------------------------------
// Device allocations go through the allocator registered with
// giamg_set_allocator, or hipMalloc / hipFree when none is.  A buffer keeps
// the allocator it came from (changing the registration later does not
// affect it) and the stream it was allocated for: the stream of the handle
// whose call allocates (AllocStreamScope), else the null stream.
struct Allocator {
    giamg_alloc_fn alloc = nullptr;     // null: hipMalloc / hipFree
    giamg_release_fn release = nullptr;
    void* ctx = nullptr;
};
Allocator registered_allocator();
hipStream_t alloc_stream();
class AllocStreamScope {
public:
    explicit AllocStreamScope(hipStream_t s);
    ~AllocStreamScope();
    AllocStreamScope(const AllocStreamScope&) = delete;
    AllocStreamScope& operator=(const AllocStreamScope&) = delete;
private:
    hipStream_t prev_;
};
// Throws GIAMG_ENOMEM on failure; `a` and `s` receive the allocator and
// stream to hand back to device_release.
void* device_alloc(size_t bytes, Allocator& a, hipStream_t& s);
void device_release(void* p, const Allocator& a, hipStream_t s);

// Owning device buffer; allocation failures raise GIAMG_ENOMEM.
template <typename T>
struct DevBuf {
    T* ptr = nullptr;
    size_t n = 0;
    Allocator owner;
    hipStream_t stream = nullptr;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), n(o.n), owner(o.owner), stream(o.stream) {
        o.ptr = nullptr;
        o.n = 0;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            ptr = o.ptr; n = o.n; owner = o.owner; stream = o.stream;
            o.ptr = nullptr; o.n = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        ptr = static_cast<T*>(device_alloc(count * sizeof(T), owner, stream));
        n = count;
    }
    void release() {
        if (ptr) device_release(ptr, owner, stream);
        ptr = nullptr;
        n = 0;
    }
    T* get() const { return ptr; }
};

// Host-side CSR (setup work).
struct HostCSR {
    int64_t nrows = 0, ncols = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> val;
    int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

// Row blocks of the streaming product for one capacity (nonzeros per block):
// bounds, descriptors and the staged-gather tables (per row block, the
// distinct columns its nonzeros touch, as runs of consecutive columns that
// the product loads into LDS first).
struct RowBlocks {
    int cap = 0;              // nonzeros per block at most
    int threads = 0;          // threads of the product kernel: rows and staged runs per block at most
    DevBuf<int64_t> rblk;     // [nblk + 1] first row of each block
    DevBuf<int64_t> bdesc;    // [4 * nblk] BlockDesc records
    int64_t nblk = 0;
    DevBuf<int32_t> run_ptr;  // [nblk + 1] offsets into runs; a block with 0 runs gathers directly
    DevBuf<int32_t> runs;     // [2 * nruns] (first column, LDS slot | length << 16)
    DevBuf<uint16_t> slot;    // [nnz] LDS slot of each nonzero's column within its block
    int64_t nruns = 0, nnz_staged = 0;
    void release_staging() {
        run_ptr.release();
        runs.release();
        slot.release();
        nruns = nnz_staged = 0;
    }
    int64_t device_bytes() const {
        return (int64_t)(rblk.n + bdesc.n) * 8 + (int64_t)(run_ptr.n + runs.n) * 4 + (int64_t)slot.n * 2;
    }
};

// Device CSR: int64 row pointers, int32 ascending columns, FP64 values and an
// optional FP32 copy of the values sharing the same index arrays.  The FP32
// products use blocks of twice the nonzeros (the same LDS bytes).
struct DevCSR {
    int64_t nrows = 0, ncols = 0, nnz = 0;
    DevBuf<int64_t> rp;
    DevBuf<int32_t> ci;
    DevBuf<double> val;
    DevBuf<float> val32;
    int lanes = 16;           // lanes per row of the row sums (mean row length)
    RowBlocks blk;            // FP64 products: 8192 nonzeros and 1024 rows per block at most
    RowBlocks blk32;          // FP32 products: 8192 nonzeros and 512 rows per block at most (val32)
    // Grouped form: rows with identical column lists share one list of LDS
    // slots (a group, at most 8 rows); a block holds groups of one size g and
    // stores its values as g planes (plane i: row i of every group, entry by
    // entry).  gnblk == 0: not built.  Layout in kernels.h (GBlock).
    int64_t gnblk = 0, gentries = 0, ggroups = 0, gnruns = 0;
    DevBuf<int64_t> gblk;     // [4 * (gnblk + 1)] GBlock records
    DevBuf<int32_t> grows;    // [nrows] rows, block by block, group by group
    DevBuf<uint32_t> ggrp;    // [ggroups] local entry offset << 16 | entries
    DevBuf<uint16_t> gslot;   // [gentries]
    DevBuf<int32_t> grun_ptr; // [gnblk + 1]
    DevBuf<int32_t> gruns;    // [2 * gnruns]
    DevBuf<double> gval;      // [nnz]
    DevBuf<float> gval32;     // [nnz] (mixed precision)
    // Lean form: small operators (at most giamg_opts.lean_max_nnz nonzeros,
    // no row longer than 8192) run a kernel that reads rows straight from
    // memory in blocks of LEAN_THREADS / lanes rows; no staging tables.
    bool lean = false;
    int64_t lean_nblk = 0;
    void release_grouping() {
        gnblk = gentries = ggroups = gnruns = 0;
        gblk.release(); grows.release(); ggrp.release(); gslot.release();
        grun_ptr.release(); gruns.release(); gval.release(); gval32.release();
    }
};
// Build the FP64 row blocks of d (and its lanes) from a host copy of its row
// pointers; setup_row_blocks32 builds the FP32 ones.
void setup_row_blocks(DevCSR& d, const std::vector<int64_t>& rp, hipStream_t s);
void setup_row_blocks32(DevCSR& d, const std::vector<int64_t>& rp, hipStream_t s);

// ---- the hierarchy ----------------------------------------------------------
struct BatchState;                 // batched-solve workspace (batch.hip)
struct BatchDeleter {
    void operator()(BatchState* b) const;
};
struct Level {
    int kind = GIAMG_LEVEL_P;
    int order = 1;
    bool device_assembled = false;  // fine level: A built by assemble_fine_device
    int64_t n = 0;
    DevCSR A, P, R;                // P, R empty on the coarsest level
    DevCSR AP;                     // A P (rows of this level, columns of the next), kept
                                   // from the Galerkin product for the post-smoothing residual
    DevBuf<double> dinv;
    DevBuf<float> dinv32;
    double lam_hat = 0.0;
    // work vectors (FP64 and FP32 sets)
    DevBuf<double> f, x, r, d0, d1, t;
    DevBuf<float> f32, x32, r32, d032, d132, t32;
    // host-side metadata for introspection
    std::vector<int32_t> l2g;      // p-levels: [n_elem][(order+1)^3], -1 = constrained
    std::vector<int32_t> agg;      // aggregates of this level's rows (if the next level is h)
};

struct Handle {
    hipStream_t stream = nullptr;
    giamg_opts opts{};
    int porder = 1;
    double lambda = 0.0;
    int64_t n_nodes = 0, n_elem = 0;
    std::vector<Level> levels;
    std::vector<uint8_t> constrained;
    // geometry kept for the load-vector helpers
    std::vector<double> corners;      // [n_elem][8][3]
    std::vector<int32_t> l2g;         // fine element map
    // coarsest level: dense inverse (FP64), rows nc
    int64_t nc = 0;
    DevBuf<double> coarse_inv;
    // PCG state (FP64)
    DevBuf<double> x, r, z, p, q, rold, tmp;
    DevBuf<double> partial;           // block partial sums
    DevBuf<double> scal;              // device scalars, see Scalars in solve.hip
    double* host_scal = nullptr;      // pinned host mirror
    DevBuf<int> ctl;                  // CG control block (stop flag, iterations, cap)
    int* host_ctl = nullptr;          // pinned host mirror
    int last_iters = 0;               // iterations of the previous solve (chunk size hint)
    // one CG iteration captured as a graph (on gstream, iterate in x), made
    // at the first solve; part1/part2: algorithmic bytes of its two halves
    hipStream_t gstream = nullptr;
    hipGraph_t it_graph = nullptr;
    hipGraphExec_t it_exec = nullptr;
    double it_part1 = 0.0, it_part2 = 0.0;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int64_t partial_cap = 0;
    // batched state
    std::unique_ptr<BatchState, BatchDeleter> batch;
    double bytes = 0.0;               // algorithmic bytes of launched kernels
    double setup_ms[7] = {0, 0, 0, 0, 0, 0, 0};
    // phase profiling (giamg_profile_enable): event intervals per category,
    // tagged with the CG iteration and half they belong to, so work queued
    // past convergence can be dropped when the solve's count is known
    struct ProfRec {
        int cat, iter, half;           // half 0: start-up or whole iteration, 1: product and
        hipEvent_t a, b;               // update, 2: V-cycle, dots and direction
    };
    struct Profile {
        int on = 0;                    // 1: every phase, 2: the fine Chebyshev step only
        int iter = 0, half = 0;        // where the host is queueing
        std::vector<hipEvent_t> pool;  // events free for reuse
        std::vector<ProfRec> pending;
        giamg_profile acc{};
    } prof;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    ~Handle();
};

// ---- host setup (setup_host.cpp) -------------------------------------------
void gll_points(int p, std::vector<double>& x, std::vector<double>& w);
void gauss_points(int m, std::vector<double>& x, std::vector<double>& w);
double lagrange_value(const std::vector<double>& nodes, int i, double x);
double lagrange_derivative(const std::vector<double>& nodes, int i, double x);

// basis: GIAMG_BASIS_NODAL or GIAMG_BASIS_MODAL (local ordering and 1-D modes)
std::vector<uint8_t> boundary_mask(const int32_t* l2g, int64_t n_elem, int p, int64_t n_nodes,
                                   int basis);
void element_corners(const double* coords, const int32_t* l2g, int64_t n_elem, int p,
                     std::vector<double>& corners, int basis);
HostCSR assemble_fine(const std::vector<double>& corners, const int32_t* l2g, int64_t n_elem,
                      int p, int64_t n_nodes, double lambda,
                      const std::vector<uint8_t>& constrained, int basis);
// 1-D tables of the element integrals: L[i][q], D[i][q] (the p + 1 modes or
// GLL Lagrange functions and their derivatives at the p + 2 Gauss points
// g[q], weights w[q]).
void reference_tables(int p, int basis, std::vector<double>& L, std::vector<double>& D,
                      std::vector<double>& g, std::vector<double>& w);
// Node -> (element, local index) lists, elements ascending within a node:
// entries nstart[i] .. nstart[i + 1] - 1 of nel / nloc.  Throws GIAMG_EINVAL
// for a node of no element.
void node_elements(const int32_t* l2g, int64_t n_elem, int nl, int64_t n_nodes, std::vector<int64_t>& nstart,
                   std::vector<int32_t>& nel, std::vector<int32_t>& nloc);
struct DevCSR;
// The p-transfer P (n_fine x n_coarse) and R = P^T built on the device, with
// the maps of p_transfer_maps; the same rows and values as p_transfer.
// make32 adds FP32 values and blocks.  Throws GIAMG_ENOTSUP when a row's
// candidates exceed the kernels' LDS lists (nothing is built then).
void p_transfer_device(const std::vector<int32_t>& l2g, int64_t n_elem, int p, int q, int64_t n_fine,
                       const std::vector<uint8_t>& free_mask, std::vector<int32_t>& l2g_next,
                       int64_t& n_coarse, int basis, DevCSR& P, DevCSR& R, bool make32, hipStream_t s);
// The same operator as assemble_fine (same pattern and entries, each entry
// summed over its elements in ascending order), built on the device into d
// (rows, columns, values and the FP64 row blocks).  Throws GIAMG_ENOTSUP when
// a row's elements hold more candidate columns than the kernels' LDS lists.
void assemble_fine_device(const std::vector<double>& corners, const int32_t* l2g, int64_t n_elem, int p,
                          int64_t n_nodes, double lambda, const std::vector<uint8_t>& constrained, int basis,
                          DevCSR& d, hipStream_t s);
void quadrature_points(const std::vector<double>& corners, int64_t n_elem, int p, double* xq);
void load_vector(const std::vector<double>& corners, const int32_t* l2g, int64_t n_elem,
                 int p, int64_t n_nodes, const std::vector<uint8_t>& constrained,
                 const double* fq, double* b, int basis);

// p-transfer: returns P (n_fine x n_coarse) and fills the next l2g.
// The maps of a p-transfer (Algorithms 2-4): l2g_next of the coarse order,
// the coarse node count, and the 1-D factor I1[i][a] ((p + 1) x (q + 1)).
void p_transfer_maps(const std::vector<int32_t>& l2g, int64_t n_elem, int p, int q, int64_t n_fine,
                     const std::vector<uint8_t>& free_mask, std::vector<int32_t>& l2g_next,
                     int64_t& n_coarse, std::vector<double>& I1, int basis);
HostCSR p_transfer(const std::vector<int32_t>& l2g, int64_t n_elem, int p, int q,
                   int64_t n_fine, const std::vector<uint8_t>& free_mask,
                   std::vector<int32_t>& l2g_next, int64_t& n_coarse, int basis);
// smoothed aggregation on a host copy of A: fills agg and returns P.
HostCSR sa_transfer(const HostCSR& A, uint64_t seed, double theta, std::vector<int32_t>& agg,
                    int64_t& n_agg);
HostCSR transpose(const HostCSR& M);
// dense SPD inverse through Cholesky; returns false if not positive definite.
bool spd_inverse(const std::vector<double>& A, int64_t n, std::vector<double>& inv);

uint64_t splitmix64(uint64_t seed, uint64_t i);
// Checks of a mesh and options before a hierarchy is built (giamg_setup and
// registered server problems): throws Error(GIAMG_EINVAL, ...) on failure.
void check_setup_args(const double* coords, int64_t n_nodes, const int32_t* l2g, int64_t n_elem,
                      int32_t p, double lambda, const giamg_opts& o);
// Held while a HIP graph is captured, and by threads of the library that
// could otherwise issue synchronising calls during another thread's capture.
std::mutex& capture_mutex();
void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& fn);

// ---- device helpers (kernels_*.hip) ----------------------------------------
void upload_csr(const HostCSR& h, DevCSR& d, hipStream_t s, bool make32);
void download_csr(const DevCSR& d, HostCSR& h, hipStream_t s);
void make_fp32_values(DevCSR& d, hipStream_t s);
// C = A * B with the full symbolic structure (device SpGEMM).
void spgemm(const DevCSR& A, const DevCSR& B, DevCSR& C, hipStream_t s);

}  // namespace giamg
