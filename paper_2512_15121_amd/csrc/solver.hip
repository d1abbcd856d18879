// Hierarchy construction and the solve phase of GIAMG-PCG on one GPU.
//
// Setup (Section 2): fine assembly on the host, then level by level the
// p-transfer (Algorithms 2-4, 7) or smoothed-aggregation transfer
// (Section 2.5) on the host and the Galerkin product R (A P) on the device
// (Section 2.1), a dense inverse of the coarsest operator, and per level the
// Jacobi diagonal and the Chebyshev interval from a power iteration.
//
// Solve (Section 2.1): CG preconditioned by one V-cycle (Algorithm 1) per
// iteration, everything on the device; the host reads one small block of
// scalars per iteration for the stopping test.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>

#include "kernels.h"

namespace giamg {

namespace {
using clock_t_ = std::chrono::steady_clock;
double ms_since(clock_t_::time_point t0) {
    return std::chrono::duration<double, std::milli>(clock_t_::now() - t0).count();
}
}  // namespace

Handle::~Handle() {
    for (hipEvent_t e : prof.pool) (void)hipEventDestroy(e);
    for (const ProfRec& r : prof.pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    if (host_scal) (void)hipHostFree(host_scal);
    if (host_ctl) (void)hipHostFree(host_ctl);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (it_exec) (void)hipGraphExecDestroy(it_exec);
    if (it_graph) (void)hipGraphDestroy(it_graph);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (gstream) (void)hipStreamDestroy(gstream);
}

namespace {
// Row blocks of capacity cap, their staging tables and descriptors.
void build_row_blocks(const DevCSR& d, RowBlocks& B, int cap, int threads, const std::vector<int64_t>& rp,
                      hipStream_t s, int* lanes) {
    std::vector<int64_t> blocks;
    int l = 16;
    make_row_blocks(rp.data(), d.nrows, cap, threads, blocks, l);
    if (lanes) *lanes = l;
    B.cap = cap;
    B.threads = threads;
    B.nblk = (int64_t)blocks.size() - 1;
    B.rblk.alloc(blocks.size());
    GIAMG_HIP(hipMemcpyAsync(B.rblk.get(), blocks.data(), blocks.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    build_staging(d, B, rp, s);
    // block descriptors (run fields from the staging tables, if any)
    std::vector<int32_t> run_ptr;
    if (B.run_ptr.get() != nullptr) {
        run_ptr.resize((size_t)B.nblk + 1);
        GIAMG_HIP(hipMemcpyAsync(run_ptr.data(), B.run_ptr.get(), run_ptr.size() * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, s));
        GIAMG_HIP(hipStreamSynchronize(s));
    }
    std::vector<BlockDesc> desc((size_t)std::max<int64_t>(B.nblk, 1));
    for (int64_t b = 0; b < B.nblk; ++b) {
        BlockDesc& D = desc[b];
        D.r0 = blocks[b];
        D.base = rp[blocks[b]];
        D.nrows = (int32_t)(blocks[b + 1] - blocks[b]);
        D.n = (int32_t)(rp[blocks[b + 1]] - D.base);
        D.run0 = run_ptr.empty() ? 0 : run_ptr[b];
        D.nruns = run_ptr.empty() ? 0 : run_ptr[b + 1] - run_ptr[b];
    }
    B.bdesc.alloc(4 * desc.size());
    GIAMG_HIP(hipMemcpyAsync(B.bdesc.get(), desc.data(), desc.size() * sizeof(BlockDesc),
                             hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipStreamSynchronize(s));
}
}  // namespace

void setup_row_blocks(DevCSR& d, const std::vector<int64_t>& rp, hipStream_t s) {
    build_row_blocks(d, d.blk, spmv_cap<double>(), spmv_threads<double>(), rp, s, &d.lanes);
}

void setup_row_blocks32(DevCSR& d, const std::vector<int64_t>& rp, hipStream_t s) {
    build_row_blocks(d, d.blk32, spmv_cap<float>(), spmv_threads<float>(), rp, s, nullptr);
}

void upload_csr(const HostCSR& h, DevCSR& d, hipStream_t s, bool make32) {
    d.nrows = h.nrows;
    d.ncols = h.ncols;
    d.nnz = h.nnz();
    d.rp.alloc(h.nrows + 1);
    d.ci.alloc(d.nnz);
    d.val.alloc(d.nnz);
    GIAMG_HIP(hipMemcpyAsync(d.rp.get(), h.rp.data(), (h.nrows + 1) * sizeof(int64_t),
                             hipMemcpyHostToDevice, s));
    if (d.nnz) {
        GIAMG_HIP(hipMemcpyAsync(d.ci.get(), h.ci.data(), d.nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
        GIAMG_HIP(hipMemcpyAsync(d.val.get(), h.val.data(), d.nnz * sizeof(double), hipMemcpyHostToDevice, s));
    }
    setup_row_blocks(d, h.rp, s);
    if (make32) {
        make_fp32_values(d, s);
        setup_row_blocks32(d, h.rp, s);
    }
}

void download_csr(const DevCSR& d, HostCSR& h, hipStream_t s) {
    h.nrows = d.nrows;
    h.ncols = d.ncols;
    h.rp.resize(d.nrows + 1);
    h.ci.resize(d.nnz);
    h.val.resize(d.nnz);
    GIAMG_HIP(hipMemcpyAsync(h.rp.data(), d.rp.get(), (d.nrows + 1) * sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
    if (d.nnz) {
        GIAMG_HIP(hipMemcpyAsync(h.ci.data(), d.ci.get(), d.nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GIAMG_HIP(hipMemcpyAsync(h.val.data(), d.val.get(), d.nnz * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    GIAMG_HIP(hipStreamSynchronize(s));
}

// Product arguments over one operator (values in the precision of T): its
// grouped form when built (with values in that precision), else its CSR
// blocks.
template <typename T>
SpmvArgs<T> args_of(const DevCSR& M, const T* val) {
    SpmvArgs<T> a;
    a.rp = M.rp.get(); a.ci = M.ci.get(); a.val = val; a.n = M.nrows;
    a.nnz = M.nnz; a.ncols = M.ncols;
    // FP32 products use the blocks of capacity SPMV_CAP32 (spmv_cap<float>)
    const RowBlocks& B = sizeof(T) == sizeof(double) ? M.blk : M.blk32;
    a.rblk = B.rblk.get(); a.nblk = B.nblk; a.lanes = M.lanes;
    a.block_cap = B.cap; a.block_threads = B.threads;
    a.bdesc = reinterpret_cast<const BlockDesc*>(B.bdesc.get());
    a.run_ptr = B.run_ptr.get(); a.runs = B.runs.get(); a.slot = B.slot.get();
    a.nnz_staged = B.nnz_staged; a.nruns = B.nruns;
    if (M.lean) {
        a.lean = true;
        a.nblk = M.lean_nblk;
        return a;
    }
    if (sizeof(T) != sizeof(double) && M.gnblk == 0 && M.nrows > 0 && M.blk32.nblk == 0)
        throw Error(GIAMG_EINVAL, "FP32 product on an operator without FP32 row blocks");
    const T* gval = nullptr;
    if constexpr (sizeof(T) == sizeof(double)) gval = M.gval.get(); else gval = M.gval32.get();
    if (M.gnblk > 0 && gval != nullptr) {
        a.gblk = reinterpret_cast<const GBlock*>(M.gblk.get());
        a.grows = M.grows.get(); a.ggrp = M.ggrp.get(); a.gslot = M.gslot.get();
        a.grun_ptr = M.grun_ptr.get(); a.gruns = M.gruns.get(); a.gval = gval;
        a.nblk = M.gnblk; a.gentries = M.gentries; a.ggroups = M.ggroups; a.gnruns = M.gnruns;
    }
    return a;
}

// Blocks of the product form args_of picks for FP64 values (the number of
// block partials its DOT and RINIT epilogues write).
int64_t product_blocks(const DevCSR& M) { return M.lean ? M.lean_nblk : M.gnblk > 0 ? M.gnblk : M.blk.nblk; }

// Lean form for the operators with at most max_nnz nonzeros and no row longer
// than spmv_cap<double>() (their staging tables are released).
void assign_lean_forms(Handle& H, int64_t max_nnz) {
    for (Level& L : H.levels)
        for (DevCSR* M : {&L.A, &L.AP, &L.P, &L.R}) {
            M->lean = false;
            M->lean_nblk = 0;
            if (M->nrows <= 0 || M->nnz > max_nnz) continue;
            std::vector<int64_t> rp((size_t)M->nrows + 1);
            GIAMG_HIP(hipMemcpyAsync(rp.data(), M->rp.get(), rp.size() * sizeof(int64_t),
                                     hipMemcpyDeviceToHost, H.stream));
            GIAMG_HIP(hipStreamSynchronize(H.stream));
            int64_t maxlen = 0;
            for (int64_t r = 0; r < M->nrows; ++r) maxlen = std::max(maxlen, rp[r + 1] - rp[r]);
            if (maxlen > spmv_cap<double>()) continue;
            const int64_t rpb = LEAN_THREADS / M->lanes;
            M->lean = true;
            M->lean_nblk = (M->nrows + rpb - 1) / rpb;
            M->blk.release_staging();
            M->blk32.release_staging();
        }
}

// Grouped forms (groups.cpp) of the operators whose rows share column lists;
// an operator that gets one drops its CSR staging tables (its products then
// always run grouped).
void build_grouped_forms(Handle& H, bool mixed) {
    for (size_t l = 0; l + 1 < H.levels.size(); ++l) {
        Level& L = H.levels[l];
        for (DevCSR* M : {&L.A, &L.AP, &L.P, &L.R}) {
            if (M->nnz <= 0 || M->lean) continue;
            std::vector<int64_t> rp((size_t)M->nrows + 1);
            std::vector<int32_t> ci((size_t)M->nnz);
            GIAMG_HIP(hipMemcpyAsync(rp.data(), M->rp.get(), rp.size() * sizeof(int64_t),
                                     hipMemcpyDeviceToHost, H.stream));
            GIAMG_HIP(hipMemcpyAsync(ci.data(), M->ci.get(), ci.size() * sizeof(int32_t),
                                     hipMemcpyDeviceToHost, H.stream));
            GIAMG_HIP(hipStreamSynchronize(H.stream));
            if (!build_grouping(*M, rp, ci, H.stream)) continue;
            if (mixed) make_fp32_group_values(*M, H.stream);
            M->blk.release_staging();
            M->blk32.release_staging();
        }
    }
    GIAMG_HIP(hipStreamSynchronize(H.stream));
}

void make_fp32_values(DevCSR& d, hipStream_t s) {
    d.val32.alloc(d.nnz);
    launch_convert<double, float>(d.nnz, d.val.get(), d.val32.get(), s);
}

namespace {
// FP32 values and, for operators in the CSR form, the FP32 row blocks.
void make_fp32_operator(DevCSR& d, hipStream_t s) {
    make_fp32_values(d, s);
    if (d.lean || d.gnblk > 0 || d.nrows <= 0) return;
    std::vector<int64_t> rp((size_t)d.nrows + 1);
    GIAMG_HIP(hipMemcpyAsync(rp.data(), d.rp.get(), rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    setup_row_blocks32(d, rp, s);
}
}  // namespace

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
namespace {

double device_dot(Handle& H, int64_t n, const double* a, const double* b) {
    launch_dot_partial(n, a, b, H.partial.get(), H.stream);
    launch_reduce(vec_blocks(n), H.partial.get(), 0, 1, H.scal.get() + S_TMP, H.stream);
    GIAMG_HIP(hipMemcpyAsync(H.host_scal + S_TMP, H.scal.get() + S_TMP, sizeof(double),
                             hipMemcpyDeviceToHost, H.stream));
    GIAMG_HIP(hipStreamSynchronize(H.stream));
    return H.host_scal[S_TMP];
}

// lambda_max(D^-1 A) by power iteration: w = D^-1 A v, estimate ||w||/||v||,
// v <- w / ||w||.
double power_estimate(Handle& H, Level& L) {
    const int64_t n = L.n;
    DevBuf<double> v(n), w(n);
    launch_power_start(n, v.get(), H.stream);
    double lam = 0.0;
    for (int it = 0; it < H.opts.power_iters; ++it) {
        SpmvArgs<double> a = args_of<double>(L.A, L.A.val.get());
        a.v = v.get(); a.y = w.get(); a.dinv = L.dinv.get();
        launch_spmv(SPMV_DINV, a, H.stream);
        const double ww = std::sqrt(device_dot(H, n, w.get(), w.get()));
        const double vv = std::sqrt(device_dot(H, n, v.get(), v.get()));
        if (!(ww > 0.0) || !std::isfinite(ww)) throw Error(GIAMG_EINVAL, "power iteration failed");
        lam = ww / vv;
        launch_scale(n, 1.0 / ww, w.get(), v.get(), H.stream);
    }
    return lam;
}

__global__ void dinv_kernel(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const double* __restrict__ val, double* __restrict__ dinv,
                            int* __restrict__ bad) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double d = 0.0;
        for (int64_t s = rp[i]; s < rp[i + 1]; ++s)
            if (ci[s] == i) d = val[s];
        if (!(d > 0.0)) *bad = 1;
        dinv[i] = 1.0 / d;
    }
}

void alloc_level_vectors(Level& L, bool mixed) {
    const int64_t n = std::max<int64_t>(L.n, 1);
    L.f.alloc(n); L.x.alloc(n); L.r.alloc(n); L.d0.alloc(n); L.d1.alloc(n); L.t.alloc(n);
    if (mixed) {
        L.f32.alloc(n); L.x32.alloc(n); L.r32.alloc(n); L.d032.alloc(n); L.d132.alloc(n); L.t32.alloc(n);
    }
}

}  // namespace

void noalloc_scratch_init();

void build_hierarchy(Handle& H, const double* coords, const int32_t* l2g) {
    noalloc_scratch_init();
    AllocStreamScope alloc_scope(H.stream);
    const giamg_opts& o = H.opts;
    const bool mixed = o.precision == GIAMG_PREC_MIXED;
    const int64_t n = H.n_nodes, ne = H.n_elem;
    auto t_all = clock_t_::now();
    auto t0 = clock_t_::now();
    // constrained nodes
    if (o.bc == GIAMG_BC_DIRICHLET) {
        H.constrained = boundary_mask(l2g, ne, H.porder, n, o.basis);
    } else {
        H.constrained.assign(n, 0);
        H.constrained[o.pin_node] = 1;
    }
    int64_t ncons = 0;
    for (auto c : H.constrained) ncons += c;
    GIAMG_REQUIRE(H.lambda > 0.0 || ncons > 0, "lambda = 0 needs at least one constrained node");
    element_corners(coords, l2g, ne, H.porder, H.corners, o.basis);
    H.l2g.assign(l2g, l2g + ne * (int64_t)(H.porder + 1) * (H.porder + 1) * (H.porder + 1));
    H.levels.clear();
    H.levels.emplace_back();
    {
        Level& L = H.levels.back();
        L.kind = GIAMG_LEVEL_P;
        L.order = H.porder;
        L.n = n;
        L.l2g = H.l2g;
        if (o.assembly != GIAMG_ASSEMBLY_HOST) {
            try {
                assemble_fine_device(H.corners, l2g, ne, H.porder, n, H.lambda, H.constrained, o.basis, L.A,
                                     H.stream);
                L.device_assembled = true;
            } catch (const Error& e) {
                // AUTO: meshes whose rows outgrow the kernels' LDS lists go to the host
                if (e.code != GIAMG_ENOTSUP || o.assembly == GIAMG_ASSEMBLY_DEVICE) throw;
                L.A = DevCSR();
            }
        }
        if (!L.device_assembled) {
            HostCSR A0 = assemble_fine(H.corners, l2g, ne, H.porder, n, H.lambda, H.constrained, o.basis);
            upload_csr(A0, L.A, H.stream, false);
        }
    }
    H.setup_ms[0] = ms_since(t0);
    // p-levels
    std::vector<uint8_t> free_mask(n);
    // keep_boundary: constrained fine nodes pass to the coarse levels too
    for (int64_t i = 0; i < n; ++i) free_mask[i] = o.keep_boundary ? 1 : !H.constrained[i];
    int order = H.porder;
    const bool explicit_schedule = o.schedule[0] != 0;
    const bool jacobi = o.preconditioner == GIAMG_PRECOND_JACOBI;   // fine level only
    for (int step = 0; !jacobi && order > 1 && (int)H.levels.size() < o.max_levels; ++step) {
        int q;
        if (explicit_schedule) {   // the listed orders only
            if (step >= 8 || o.schedule[step] == 0) break;
            q = o.schedule[step];
        } else {                   // q = p / spf(p)
            int spf = 2;
            while (spf * spf <= order && order % spf) ++spf;
            if (order % spf) spf = order;
            q = order / spf;
        }
        t0 = clock_t_::now();
        std::vector<int32_t> l2g_next;
        int64_t nc = 0;
        Level& F = H.levels.back();
        bool on_device = false;
        if (o.assembly != GIAMG_ASSEMBLY_HOST) {
            try {
                p_transfer_device(F.l2g, ne, order, q, F.n, free_mask, l2g_next, nc, o.basis, F.P, F.R, mixed,
                                  H.stream);
                on_device = true;
            } catch (const Error& e) {
                // AUTO: rows that outgrow the kernels' LDS lists go to the host
                if (e.code != GIAMG_ENOTSUP || o.assembly == GIAMG_ASSEMBLY_DEVICE) throw;
                F.P = DevCSR();
                F.R = DevCSR();
            }
        }
        if (!on_device) {
            HostCSR P = p_transfer(F.l2g, ne, order, q, F.n, free_mask, l2g_next, nc, o.basis);
            if (nc > 0) {
                HostCSR R = transpose(P);
                upload_csr(P, F.P, H.stream, mixed);
                upload_csr(R, F.R, H.stream, mixed);
            }
        }
        H.setup_ms[1] += ms_since(t0);
        if (nc == 0) {
            F.P = DevCSR();
            F.R = DevCSR();
            break;
        }
        t0 = clock_t_::now();
        spgemm(F.A, F.P, F.AP, H.stream);
        Level C;
        C.kind = GIAMG_LEVEL_P;
        C.order = q;
        C.n = nc;
        C.l2g = std::move(l2g_next);
        spgemm(F.R, F.AP, C.A, H.stream);
        H.setup_ms[3] += ms_since(t0);
        H.levels.push_back(std::move(C));
        free_mask.assign(nc, 1);
        order = q;
    }
    // h-levels (smoothed aggregation) below order 1
    while (!jacobi && H.levels.back().order == 1 && H.levels.back().n > o.coarse_max &&
           (int)H.levels.size() < o.max_levels) {
        Level& F = H.levels.back();
        t0 = clock_t_::now();
        HostCSR Ah;
        download_csr(F.A, Ah, H.stream);
        int64_t nagg = 0;
        HostCSR P = sa_transfer(Ah, o.agg_seed, o.theta, F.agg, nagg);
        H.setup_ms[2] += ms_since(t0);
        if (nagg >= F.n || nagg == 0) {
            F.agg.clear();
            break;
        }
        HostCSR R = transpose(P);
        upload_csr(P, F.P, H.stream, mixed);
        upload_csr(R, F.R, H.stream, mixed);
        t0 = clock_t_::now();
        spgemm(F.A, F.P, F.AP, H.stream);
        Level C;
        C.kind = GIAMG_LEVEL_H;
        C.order = 1;
        C.n = nagg;
        spgemm(F.R, F.AP, C.A, H.stream);
        H.setup_ms[3] += ms_since(t0);
        H.levels.push_back(std::move(C));
    }
    // coarsest: dense inverse through Cholesky
    t0 = clock_t_::now();
    if (!jacobi) {
        Level& Lc = H.levels.back();
        H.nc = Lc.n;
        GIAMG_REQUIRE(H.nc <= 16384, "coarsest level too large for the dense solve");
        HostCSR Ah;
        download_csr(Lc.A, Ah, H.stream);
        std::vector<double> dense(H.nc * H.nc, 0.0), inv;
        for (int64_t i = 0; i < H.nc; ++i)
            for (int64_t s = Ah.rp[i]; s < Ah.rp[i + 1]; ++s) dense[i * H.nc + Ah.ci[s]] = Ah.val[s];
        if (H.nc > 0) {
            if (!spd_inverse(dense, H.nc, inv))
                throw Error(GIAMG_EINVAL, "coarsest operator is not positive definite");
            H.coarse_inv.alloc(H.nc * H.nc);
            GIAMG_HIP(hipMemcpyAsync(H.coarse_inv.get(), inv.data(), inv.size() * sizeof(double),
                                     hipMemcpyHostToDevice, H.stream));
            GIAMG_HIP(hipStreamSynchronize(H.stream));
        }
    }
    H.setup_ms[4] = ms_since(t0);
    t0 = clock_t_::now();
    if (o.lean_max_nnz > 0) assign_lean_forms(H, o.lean_max_nnz);
    if (o.row_groups && !o.direct_gathers) build_grouped_forms(H, mixed);
    const double grouping_ms = ms_since(t0);
    // work buffers
    int64_t maxn = 1, maxblk = 1;
    for (auto& L : H.levels) {
        maxn = std::max(maxn, L.n);
        for (const DevCSR* M : {&L.A, &L.P, &L.R, &L.AP})
            maxblk = std::max({maxblk, M->blk.nblk, M->blk32.nblk, M->gnblk, M->lean_nblk});
    }
    H.partial_cap = std::max<int64_t>(2 * maxblk, 2 * vec_blocks(maxn)) + 16;
    H.partial.alloc(H.partial_cap);
    H.scal.alloc(S_COUNT);
    GIAMG_HIP(hipMemsetAsync(H.scal.get(), 0, S_COUNT * sizeof(double), H.stream));
    if (!H.host_scal) GIAMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&H.host_scal), S_COUNT * sizeof(double)));
    H.ctl.alloc(C_COUNT);
    if (!H.host_ctl) GIAMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&H.host_ctl), C_COUNT * sizeof(int)));
    // smoother data
    t0 = clock_t_::now();
    for (size_t l = 0; l < H.levels.size(); ++l) {
        Level& L = H.levels[l];
        alloc_level_vectors(L, mixed);
        if (mixed) make_fp32_operator(L.A, H.stream);
        if (l + 1 == H.levels.size() && !jacobi) break;
        if (mixed) make_fp32_operator(L.AP, H.stream);
        L.dinv.alloc(L.n);
        DevBuf<int> bad(1);
        GIAMG_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), H.stream));
        dinv_kernel<<<(unsigned)std::min<int64_t>((L.n + 255) / 256, 65536), 256, 0, H.stream>>>(
            L.n, L.A.rp.get(), L.A.ci.get(), L.A.val.get(), L.dinv.get(), bad.get());
        GIAMG_HIP(hipGetLastError());
        int hbad = 0;
        GIAMG_HIP(hipMemcpyAsync(&hbad, bad.get(), sizeof(int), hipMemcpyDeviceToHost, H.stream));
        GIAMG_HIP(hipStreamSynchronize(H.stream));
        if (hbad) throw Error(GIAMG_EINVAL, "non-positive diagonal on level " + std::to_string(l));
        if (mixed) {
            L.dinv32.alloc(L.n);
            launch_convert<double, float>(L.n, L.dinv.get(), L.dinv32.get(), H.stream);
        }
        if (jacobi) break;   // the diagonal is the whole preconditioner
        L.lam_hat = power_estimate(H, L);
    }
    H.setup_ms[5] = ms_since(t0) + grouping_ms;
    const int64_t nn = std::max<int64_t>(n, 1);
    H.x.alloc(nn); H.r.alloc(nn); H.z.alloc(nn); H.p.alloc(nn); H.q.alloc(nn); H.rold.alloc(nn);
    H.tmp.alloc(nn);
    if (o.direct_gathers) {
        for (auto& L : H.levels)
            for (DevCSR* M : {&L.A, &L.P, &L.R, &L.AP}) {
                M->blk.release_staging();
                M->blk32.release_staging();
            }
    }
    if (!H.ev0) GIAMG_HIP(hipEventCreate(&H.ev0));
    if (!H.ev1) GIAMG_HIP(hipEventCreate(&H.ev1));
    if (!H.ev_fork) GIAMG_HIP(hipEventCreateWithFlags(&H.ev_fork, hipEventDisableTiming));
    if (!H.ev_join) GIAMG_HIP(hipEventCreateWithFlags(&H.ev_join, hipEventDisableTiming));
    if (!H.gstream) GIAMG_HIP(hipStreamCreateWithFlags(&H.gstream, hipStreamNonBlocking));
    GIAMG_HIP(hipStreamSynchronize(H.stream));
    H.setup_ms[6] = ms_since(t_all);
}

int64_t handle_device_bytes(const Handle& H) {
    auto csr = [](const DevCSR& m) {
        return (int64_t)m.rp.n * 8 + (int64_t)m.ci.n * 4 + (int64_t)m.val.n * 8 + (int64_t)m.val32.n * 4 +
               m.blk.device_bytes() + m.blk32.device_bytes() +
               (int64_t)m.gblk.n * 8 + (int64_t)(m.grows.n + m.ggrp.n + m.grun_ptr.n + m.gruns.n) * 4 +
               (int64_t)m.gslot.n * 2 + (int64_t)m.gval.n * 8 + (int64_t)m.gval32.n * 4;
    };
    int64_t b = 0;
    for (const Level& L : H.levels) {
        b += csr(L.A) + csr(L.P) + csr(L.R) + csr(L.AP);
        b += (int64_t)(L.dinv.n + L.f.n + L.x.n + L.r.n + L.d0.n + L.d1.n + L.t.n) * 8;
        b += (int64_t)(L.dinv32.n + L.f32.n + L.x32.n + L.r32.n + L.d032.n + L.d132.n + L.t32.n) * 4;
    }
    b += (int64_t)H.coarse_inv.n * 8;
    b += (int64_t)(H.x.n + H.r.n + H.z.n + H.p.n + H.q.n + H.rold.n + H.tmp.n + H.partial.n) * 8;
    return b;
}

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------
namespace {

template <typename T> struct LV;
template <> struct LV<double> {
    static const double* A(const Level& L) { return L.A.val.get(); }
    static const double* P(const Level& L) { return L.P.val.get(); }
    static const double* R(const Level& L) { return L.R.val.get(); }
    static const double* AP(const Level& L) { return L.AP.val.get(); }
    static const double* dinv(const Level& L) { return L.dinv.get(); }
    static double* f(Level& L) { return L.f.get(); }
    static double* x(Level& L) { return L.x.get(); }
    static double* r(Level& L) { return L.r.get(); }
    static double* d0(Level& L) { return L.d0.get(); }
    static double* d1(Level& L) { return L.d1.get(); }
    static double* t(Level& L) { return L.t.get(); }
};
template <> struct LV<float> {
    static const float* A(const Level& L) { return L.A.val32.get(); }
    static const float* P(const Level& L) { return L.P.val32.get(); }
    static const float* R(const Level& L) { return L.R.val32.get(); }
    static const float* AP(const Level& L) { return L.AP.val32.get(); }
    static const float* dinv(const Level& L) { return L.dinv32.get(); }
    static float* f(Level& L) { return L.f32.get(); }
    static float* x(Level& L) { return L.x32.get(); }
    static float* r(Level& L) { return L.r32.get(); }
    static float* d0(Level& L) { return L.d032.get(); }
    static float* d1(Level& L) { return L.d132.get(); }
    static float* t(Level& L) { return L.t32.get(); }
};

template <typename T>
SpmvArgs<T> args_A(const Level& L) {
    SpmvArgs<T> a = args_of<T>(L.A, LV<T>::A(L));
    a.dinv = LV<T>::dinv(L);
    return a;
}

// Algorithmic HBM bytes of one product launch: values, column ids (16-bit
// slots plus the run tables in staged blocks), row pointers, the gathered
// vector once, and the row-local vectors its epilogue reads and writes.
template <typename T>
double spmv_bytes(int mode, const SpmvArgs<T>& a) {
    const double vb = sizeof(T);
    double rows = 0;
    switch (mode) {
        case SPMV_PLAIN: rows = 1; break;             // y
        case SPMV_RESID: rows = 2; break;             // f, y
        case SPMV_ADD: rows = 2; break;               // y read + write
        case SPMV_CHEB_INIT: rows = 4; break;         // f, dinv, r, d_new
        case SPMV_CHEB_STEP: rows = (a.flags & CHEB_ASSIGN) ? 5 : 6; break;  // r rw, dinv, d_new, x (r)w
        case SPMV_JACOBI: rows = 3; break;            // f, dinv, y
        case SPMV_DOT: rows = 1; break;               // y
        case SPMV_DINV: rows = 2; break;              // dinv, y
        case SPMV_RINIT: rows = 2; break;             // f, y
        case SPMV_RCHEB0: rows = 4; break;            // dinv, y, r, d_0
    }
    if (a.gblk != nullptr)   // grouped: slots per entry, block records, row list, group table
        return vb * a.nnz + 2.0 * a.gentries + 8.0 * a.gnruns + (4.0 + 32.0) * (a.nblk + 1) + 4.0 * a.n +
               4.0 * a.ggroups + vb * a.ncols + rows * vb * a.n;
    const double staged = a.run_ptr ? 2.0 * a.nnz_staged + 8.0 * a.nruns + 4.0 * (a.nblk + 1) : 0.0;
    return vb * a.nnz + 4.0 * (a.nnz - a.nnz_staged) + staged + 8.0 * (a.n + 1) + vb * a.ncols +
           rows * vb * a.n;
}

// ---- phase profiling -------------------------------------------------------
hipEvent_t prof_event(Handle& H) {
    if (!H.prof.pool.empty()) {
        hipEvent_t e = H.prof.pool.back();
        H.prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    GIAMG_HIP(hipEventCreate(&e));
    return e;
}

// Events around one phase on the handle's stream while profiling is on.
class Phase {
public:
    Phase(Handle& h, int cat) : H(h), cat_(cat) {
        if (H.prof.on != 1 || cat < 0) return;
        a_ = prof_event(H);
        GIAMG_HIP(hipEventRecord(a_, H.stream));
    }
    ~Phase() {
        if (a_ == nullptr) return;
        hipEvent_t b = nullptr;
        if (!H.prof.pool.empty()) {
            b = H.prof.pool.back();
            H.prof.pool.pop_back();
        } else if (hipEventCreate(&b) != hipSuccess) {
            b = nullptr;
        }
        try {
            if (b != nullptr && hipEventRecord(b, H.stream) == hipSuccess) {
                H.prof.pending.push_back({cat_, H.prof.iter, H.prof.half, a_, b});
                return;
            }
        } catch (...) {
        }
        (void)hipEventDestroy(a_);
        if (b != nullptr) (void)hipEventDestroy(b);
    }
    Phase(const Phase&) = delete;
    Phase& operator=(const Phase&) = delete;

private:
    Handle& H;
    int cat_;
    hipEvent_t a_ = nullptr;
};

// Sum the intervals of a finished solve: iters CG iterations, whose first
// halves (product, update, stopping test) ran for iterations 1..first and
// second halves (V-cycle, dots, direction) for 1..second.
void prof_harvest(Handle& H, int iters, int first, int second) {
    for (const Handle::ProfRec& r : H.prof.pending) {
        const bool ran = r.iter == 0 || (r.half == 2 ? r.iter <= second : r.iter <= first);
        if (ran) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                H.prof.acc.ms[r.cat] += t;
                H.prof.acc.count[r.cat] += 1;
            }
        }
        H.prof.pool.push_back(r.a);
        H.prof.pool.push_back(r.b);
    }
    H.prof.pending.clear();
    H.prof.acc.solves += 1;
    H.prof.acc.iterations += iters;
}

template <typename T>
void run_spmv(Handle& H, int mode, const SpmvArgs<T>& a) {
    H.bytes += spmv_bytes(mode, a);
    launch_spmv(mode, a, H.stream);
}

struct ChebCoef {
    double inv_theta;
    std::vector<double> c1, c2;   // per step j = 1..k-1
};

ChebCoef cheb_coef(const Handle& H, const Level& L) {
    const double lo = H.opts.cheb_lo * L.lam_hat, hi = H.opts.cheb_hi * L.lam_hat;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    ChebCoef c;
    c.inv_theta = 1.0 / theta;
    double rho = 1.0 / sigma;
    for (int j = 1; j < H.opts.degree; ++j) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        c.c1.push_back(rn * rho);
        c.c2.push_back(2.0 * rn / delta);
        rho = rn;
    }
    return c;
}


// Chebyshev acceleration of Jacobi (Saad, Algorithm 12.1, on D^-1 A):
//   r_0 = D^-1 (f - A x_0), d_0 = r_0 / theta,
//   x_{j+1} = x_j + d_j,
//   r_{j+1} = r_j - D^-1 A d_j,
//   d_{j+1} = rho_{j+1} rho_j d_j + (2 rho_{j+1} / delta) r_{j+1}.
// The update of x by d_j is deferred into the next product's epilogue (the
// product gathers d, never x), so no kernel reads and writes x at once.
// zero_start: pre-smoothing from x = 0 (x is not read); init_done: the
// kernel that produced f already wrote r_0 and d_0 (fused_init_ok).
// Post-smoothing after a coarse correction x = x' + P e may pass the residual
// t = f - A x' from before the correction and the coarse vector e: then
// f - A x = t - (A P) e, a product with A P, whose rows are several times
// shorter than those of A on the p-levels.
template <typename T>
void smooth_chebyshev(Handle& H, Level& L, const T* f, T* x, bool zero_start,
                      const T* t = nullptr, const T* e = nullptr, bool init_done = false) {
    const int k = H.opts.degree;
    const ChebCoef c = cheb_coef(H, L);
    T* r = LV<T>::r(L);
    T* d[2] = {LV<T>::d0(L), LV<T>::d1(L)};
    if (zero_start) {
        if (!init_done) {
            H.bytes += (k == 1 ? 5.0 : 4.0) * sizeof(T) * L.n;
            launch_cheb_init0<T>(L.n, f, LV<T>::dinv(L), r, d[0], x, (T)c.inv_theta, k == 1, H.stream);
        }
    } else if (e != nullptr) {
        SpmvArgs<T> a = args_of<T>(L.AP, LV<T>::AP(L));
        a.dinv = LV<T>::dinv(L);
        a.v = e; a.f = t; a.r = r; a.y = d[0]; a.inv_theta = (T)c.inv_theta;
        run_spmv(H, SPMV_CHEB_INIT, a);
        if (k == 1) {
            H.bytes += 3.0 * sizeof(T) * L.n;
            launch_add<T>(L.n, d[0], x, H.stream);
        }
    } else {
        SpmvArgs<T> a = args_A<T>(L);
        a.v = x; a.f = f; a.r = r; a.y = d[0]; a.inv_theta = (T)c.inv_theta;
        run_spmv(H, SPMV_CHEB_INIT, a);
        if (k == 1) {
            H.bytes += 3.0 * sizeof(T) * L.n;
            launch_add<T>(L.n, d[0], x, H.stream);
        }
    }
    for (int j = 1; j < k; ++j) {
        SpmvArgs<T> a = args_A<T>(L);
        a.v = d[(j - 1) & 1]; a.y = d[j & 1]; a.r = r; a.x = x;
        a.c1 = (T)c.c1[j - 1]; a.c2 = (T)c.c2[j - 1];
        a.flags = (j == k - 1 ? CHEB_LAST : 0) | ((zero_start && j == 1) ? CHEB_ASSIGN : 0);
        if (H.prof.on != 0 && &L == &H.levels[0]) {   // the dominant kernel, timed by its dispatch
            a.ev_start = prof_event(H);
            a.ev_stop = prof_event(H);
            H.prof.pending.push_back({GIAMG_PHASE_FINE_STEP, H.prof.iter, H.prof.half, a.ev_start,
                                      a.ev_stop});
        }
        run_spmv(H, SPMV_CHEB_STEP, a);
    }
}

// Fused inits for the Chebyshev smoother with degree >= 2: the restriction
// writes the next level's r_0, d_0 and the CG update the fine level's (the
// same operations as cheb_init0_kernel, so the same bits).
bool fused_init_ok(const Handle& H) {
    return H.opts.smoother == GIAMG_SMOOTHER_CHEBYSHEV && H.opts.degree >= 2;
}

// Weighted Jacobi x <- x + omega D^-1 (f - A x), ping-pong between x and d0.
template <typename T>
void smooth_jacobi(Handle& H, Level& L, const T* f, T* x, bool zero_start) {
    const int sweeps = H.opts.degree;
    const T w = (T)H.opts.omega;
    T* buf[2] = {x, LV<T>::d0(L)};
    int cur = 0, start = 0;
    if (zero_start) {
        H.bytes += 3.0 * sizeof(T) * L.n;
        launch_jacobi0<T>(L.n, f, LV<T>::dinv(L), x, w, H.stream);
        start = 1;
    }
    for (int s = start; s < sweeps; ++s) {
        SpmvArgs<T> a = args_A<T>(L);
        a.v = buf[cur]; a.y = buf[1 - cur]; a.f = f; a.omega = w;
        run_spmv(H, SPMV_JACOBI, a);
        cur = 1 - cur;
    }
    if (cur == 1) {
        H.bytes += 2.0 * sizeof(T) * L.n;
        launch_copy<T>(L.n, buf[1], x, H.stream);
    }
}

template <typename T>
void smooth(Handle& H, Level& L, const T* f, T* x, bool zero_start, const T* t = nullptr,
            const T* e = nullptr, bool init_done = false) {
    if (H.opts.smoother == GIAMG_SMOOTHER_CHEBYSHEV)
        smooth_chebyshev<T>(H, L, f, x, zero_start, t, e, init_done);
    else
        smooth_jacobi<T>(H, L, f, x, zero_start);
}

template <typename T>
void residual(Handle& H, Level& L, const T* f, const T* x, T* out) {
    SpmvArgs<T> a = args_A<T>(L);
    a.v = x; a.f = f; a.y = out;
    run_spmv(H, SPMV_RESID, a);
}

template <typename T>
void restrict_to(Handle& H, Level& L, const T* r, T* fc) {
    SpmvArgs<T> a = args_of<T>(L.R, LV<T>::R(L));
    a.v = r; a.y = fc;
    run_spmv(H, SPMV_PLAIN, a);
}

// Restriction fused with the zero-start Chebyshev init of level C.
template <typename T>
void restrict_cheb0(Handle& H, Level& L, Level& C, const T* r) {
    SpmvArgs<T> a = args_of<T>(L.R, LV<T>::R(L));
    a.v = r; a.y = LV<T>::f(C); a.dinv = LV<T>::dinv(C);
    a.r = LV<T>::r(C); a.x = LV<T>::d0(C);
    a.inv_theta = (T)cheb_coef(H, C).inv_theta;
    run_spmv(H, SPMV_RCHEB0, a);
}

template <typename T>
void prolong_add(Handle& H, Level& L, const T* ec, T* x) {
    SpmvArgs<T> a = args_of<T>(L.P, LV<T>::P(L));
    a.v = ec; a.y = x;
    run_spmv(H, SPMV_ADD, a);
}

// Algorithm 1: one V-cycle from level l for right-hand side f, result in x.
// init_done: level l's zero-start smoother init was written with f (fused).
template <typename T>
void vcycle(Handle& H, size_t l, const T* f, T* x, bool init_done = false) {
    Level& L = H.levels[l];
    if (l + 1 == H.levels.size()) {
        Phase ph(H, GIAMG_PHASE_COARSE);
        H.bytes += 8.0 * H.nc * H.nc + 2.0 * sizeof(T) * H.nc;
        launch_coarse_apply<T>(H.nc, H.coarse_inv.get(), f, x, H.stream);
        return;
    }
    Level& C = H.levels[l + 1];
    {
        Phase ph(H, GIAMG_PHASE_SMOOTH);
        Phase ph0(H, l == 0 ? GIAMG_PHASE_FIRST_SMOOTH : -1);
        smooth<T>(H, L, f, x, true, nullptr, nullptr, init_done);
    }
    {
        Phase ph(H, GIAMG_PHASE_RESIDUAL);
        residual<T>(H, L, f, x, LV<T>::t(L));
    }
    const bool fuse = fused_init_ok(H) && l + 2 < H.levels.size();
    {
        Phase ph(H, GIAMG_PHASE_TRANSFER);
        if (fuse)
            restrict_cheb0<T>(H, L, C, LV<T>::t(L));
        else
            restrict_to<T>(H, L, LV<T>::t(L), LV<T>::f(C));
    }
    vcycle<T>(H, l + 1, LV<T>::f(C), LV<T>::x(C), fuse);
    {
        Phase ph(H, GIAMG_PHASE_TRANSFER);
        prolong_add<T>(H, L, LV<T>::x(C), x);
    }
    Phase ph(H, GIAMG_PHASE_SMOOTH);
    Phase ph0(H, l == 0 ? GIAMG_PHASE_FIRST_SMOOTH : -1);
    smooth<T>(H, L, f, x, false, LV<T>::t(L), LV<T>::x(C));
}

// z = V-cycle(r).  init_done: the fine level's smoother init was fused into
// the CG update.  Mixed precision: the FP32 cycle runs from level 0's f32
// (r rounded; r32_ready: the CG update wrote it) and z stays in FP32 in
// level 0's x32 (zvec32), read by the dots and the direction update widened
// exactly; z is not written.
void precondition(Handle& H, const double* r, double* z, bool init_done = false, bool r32_ready = false) {
    if (H.opts.preconditioner == GIAMG_PRECOND_JACOBI) {   // z = D^-1 r
        Level& L = H.levels[0];
        H.bytes += 24.0 * L.n;
        launch_mul(L.n, L.dinv.get(), r, z, H.stream);
        return;
    }
    Phase ph(H, GIAMG_PHASE_VCYCLE);
    if (H.opts.precision == GIAMG_PREC_MIXED) {
        Level& L = H.levels[0];
        if (!r32_ready) {
            H.bytes += 12.0 * L.n;
            launch_convert<double, float>(L.n, r, L.f32.get(), H.stream);
        }
        vcycle<float>(H, 0, L.f32.get(), L.x32.get(), init_done);
    } else {
        vcycle<double>(H, 0, r, z, init_done);
    }
}

const float* zvec32(Handle& H) { return H.levels[0].x32.get(); }

// Points the handle's stream at another one for the scope (graph capture).
struct StreamSwap {
    Handle& H;
    hipStream_t saved;
    StreamSwap(Handle& h, hipStream_t st) : H(h), saved(h.stream) { H.stream = st; }
    ~StreamSwap() { H.stream = saved; }
};

void fetch_scalars(Handle& H, const double* scal) {
    GIAMG_HIP(hipMemcpyAsync(H.host_scal, scal, S_COUNT * sizeof(double),
                             hipMemcpyDeviceToHost, H.stream));
    GIAMG_HIP(hipStreamSynchronize(H.stream));
}

}  // namespace

// ---------------------------------------------------------------------------
// CG preconditioned by the V-cycle
// ---------------------------------------------------------------------------
namespace {
// Device memory the solve works in besides the hierarchy: the iterate, the
// CG vectors, block partial sums, device scalars and the control block.
struct CgWork {
    double *x, *r, *z, *p, *q, *rold, *tmp, *partial, *scal;
    int* ctl;
};

// allow_graph: with graph_launch one iteration may be captured (the handle's
// work buffers only: the captured pointers must stay valid for the handle).
int solve_on(Handle& H, const CgWork& w, bool allow_graph, const double* b, double* x, double tol,
             giamg_info* info) {
    AllocStreamScope alloc_scope(H.stream);
    const int64_t n = H.n_nodes;
    const Level& L0 = H.levels[0];
    const bool flexible = H.opts.precision == GIAMG_PREC_MIXED;
    hipStream_t s = H.stream;
    const int64_t gs = product_blocks(L0.A), gv = vec_blocks(n);
    // initial: a zero guess (flagged on the device) skips the product; at
    // exit the true residual of the solution is always formed
    auto rinit = [&](double* out, bool initial) {
        SpmvArgs<double> a = args_of<double>(L0.A, L0.A.val.get());
        a.v = x; a.f = b; a.y = out; a.partial = w.partial;
        if (initial) a.vnz = w.scal + S_XNZ;
        run_spmv(H, SPMV_RINIT, a);
    };
    H.bytes = 0.0;
    H.prof.iter = 0;
    H.prof.half = 0;
    GIAMG_HIP(hipEventRecord(H.ev0, s));
    launch_fill(S_COUNT, 0.0, w.scal, s);
    launch_nonzero_flag(n, x, w.scal + S_XNZ, s);
    rinit(w.r, true);
    launch_reduce(gs, w.partial, gs, 2, w.scal + S_BB, s);
    fetch_scalars(H, w.scal);
    const double bnorm = std::sqrt(H.host_scal[S_BB]);
    int status = GIAMG_OK;
    int iters = 0;
    int prof_first = 0, prof_second = 0;   // CG halves that ran (profiling)
    double relres = 0.0;
    if (bnorm == 0.0) {
        H.bytes += 8.0 * n;
        launch_fill(n, 0.0, x, s);
    } else {
        relres = std::sqrt(H.host_scal[S_RR]) / bnorm;
        if (!(relres < tol) && H.opts.maxit > 0) {
            // device-side convergence test: tolerance and control block
            H.host_scal[S_TOL] = tol;
            GIAMG_HIP(hipMemcpyAsync(w.scal + S_TOL, H.host_scal + S_TOL, sizeof(double),
                                     hipMemcpyHostToDevice, s));
            H.host_ctl[C_STOP] = 0;
            H.host_ctl[C_ITERS] = 0;
            H.host_ctl[C_MAXIT] = H.opts.maxit;
            H.host_ctl[3] = 0;
            GIAMG_HIP(hipMemcpyAsync(w.ctl, H.host_ctl, C_COUNT * sizeof(int), hipMemcpyHostToDevice, s));
            precondition(H, w.r, w.z);
            if (flexible) {
                H.bytes += 32.0 * n;
                launch_dot_partial(n, w.r, zvec32(H), w.partial, s);
                launch_reduce(gv, w.partial, 0, 1, w.scal + S_RZNEW, s, FIN_BETA_FIRST,
                              w.scal);
                launch_convert<float, double>(n, zvec32(H), w.p, s);
            } else {
                H.bytes += 32.0 * n;
                launch_dot_partial(n, w.r, w.z, w.partial, s);
                launch_reduce(gv, w.partial, 0, 1, w.scal + S_RZNEW, s, FIN_BETA_FIRST,
                              w.scal);
                launch_copy<double>(n, w.z, w.p, s);
            }
            // Iterations are queued in chunks without reading anything back:
            // the reduction that closes an iteration sets the device stop
            // flag, after which every queued kernel returns at once.  The
            // host reads the control block between chunks only; the first
            // chunk is the previous solve's iteration count.  With
            // graph_launch one iteration is a graph, captured at the first
            // solve of the handle and replayed on the handle's graph stream.
            // The iterate lives in the handle's x (copied in and out), so the
            // graph's pointers never change.
            const bool graph = allow_graph && H.opts.graph_launch != 0 && H.prof.on == 0;
            // Chebyshev smoother of degree >= 2: the fine level's smoother
            // init rides on the CG update (bitwise the same vectors; FP32 in
            // mixed precision)
            const bool fused = fused_init_ok(H) && H.levels.size() > 1;
            double* xi = w.x;
            H.bytes += 16.0 * n;
            launch_copy<double>(n, x, xi, s);
            auto iteration = [&]() {
                hipStream_t st = H.stream;
                const double b0 = H.bytes;
                Phase pcg(H, GIAMG_PHASE_PCG);
                H.prof.half = 1;
                {
                    Phase ph(H, GIAMG_PHASE_CG_MATVEC);
                    SpmvArgs<double> a = args_of<double>(L0.A, L0.A.val.get());
                    a.v = w.p; a.y = w.q; a.partial = w.partial;
                    H.bytes += (flexible ? 56.0 : 48.0) * n;
                    run_spmv(H, SPMV_DOT, a);
                }
                {
                    Phase ph(H, GIAMG_PHASE_CG_DOT);
                    launch_reduce(gs, w.partial, 0, 1, w.scal + S_PQ, st, FIN_ALPHA, w.scal);
                }
                {
                    Phase ph(H, GIAMG_PHASE_CG_UPDATE);
                    if (flexible) {   // also r in FP32 (and level 0's FP32 Chebyshev r_0, d_0)
                        Level& F = H.levels[0];
                        H.bytes += (fused ? 16.0 : 4.0) * n;
                        launch_pcg_update_mixed(n, xi, w.r, w.rold, w.p, w.q,
                                                w.scal, w.partial, F.f32.get(),
                                                fused ? F.dinv32.get() : nullptr, F.r32.get(),
                                                F.d032.get(), (float)cheb_coef(H, F).inv_theta, st);
                    } else if (fused) {   // the update also writes level 0's Chebyshev r_0, d_0
                        Level& F = H.levels[0];
                        H.bytes += 24.0 * n;
                        launch_pcg_update_cheb0(n, xi, w.r, w.p, w.q, w.scal,
                                                w.partial, F.dinv.get(), F.r.get(), F.d0.get(),
                                                cheb_coef(H, F).inv_theta, st);
                    } else {
                        launch_pcg_update(n, xi, w.r, flexible ? w.rold : nullptr, w.p,
                                          w.q, w.scal, w.partial, st);
                    }
                }
                {
                    Phase ph(H, GIAMG_PHASE_CG_DOT);
                    launch_reduce(gv, w.partial, 0, 1, w.scal + S_RR, st, FIN_CONV,
                                  w.scal, w.ctl);
                }
                const double b1 = H.bytes;
                H.prof.half = 2;
                precondition(H, w.r, w.z, fused, flexible);
                if (flexible) {
                    {
                        Phase ph(H, GIAMG_PHASE_CG_DOT);
                        H.bytes += 20.0 * n;
                        launch_dot2_partial(n, w.r, zvec32(H), w.rold, w.partial, st);
                        launch_reduce(gv, w.partial, gv, 2, w.scal + S_RZNEW, st, FIN_BETA_FLEX,
                                      w.scal);
                    }
                    Phase ph(H, GIAMG_PHASE_CG_UPDATE);
                    H.bytes += 20.0 * n;
                    launch_pcg_direction(n, zvec32(H), w.p, w.scal, st);
                } else {
                    {
                        Phase ph(H, GIAMG_PHASE_CG_DOT);
                        H.bytes += 16.0 * n;
                        launch_dot_partial(n, w.r, w.z, w.partial, st);
                        launch_reduce(gv, w.partial, 0, 1, w.scal + S_RZNEW, st, FIN_BETA,
                                      w.scal);
                    }
                    Phase ph(H, GIAMG_PHASE_CG_UPDATE);
                    H.bytes += 24.0 * n;
                    launch_pcg_direction(n, w.z, w.p, w.scal, st);
                }
                H.prof.half = 0;
                H.it_part1 = b1 - b0;
                H.it_part2 = H.bytes - b1;
            };
            hipStream_t its = s;
            if (graph) {
                its = H.gstream;
                if (!H.it_exec) {
                    const double keep = H.bytes;
                    StreamSwap swap(H, its);
                    StopScope scope(w.ctl);
                    std::lock_guard<std::mutex> cap(capture_mutex());
                    GIAMG_HIP(hipStreamBeginCapture(its, hipStreamCaptureModeRelaxed));
                    try {
                        iteration();
                    } catch (...) {
                        hipGraph_t g = nullptr;
                        (void)hipStreamEndCapture(its, &g);
                        if (g) (void)hipGraphDestroy(g);
                        throw;
                    }
                    GIAMG_HIP(hipStreamEndCapture(its, &H.it_graph));
                    GIAMG_HIP(hipGraphInstantiate(&H.it_exec, H.it_graph, nullptr, nullptr, 0));
                    H.bytes = keep;
                }
                GIAMG_HIP(hipEventRecord(H.ev_fork, s));
                GIAMG_HIP(hipStreamWaitEvent(its, H.ev_fork, 0));
            }
            const double bytes0 = H.bytes;
            int launched = 0;
            int chunk = H.last_iters > 0 ? H.last_iters : 8;
            {
                StopScope scope(w.ctl);
                for (;;) {
                    const int todo = std::min(chunk, H.opts.maxit - launched);
                    for (int j = 0; j < todo; ++j) {
                        H.prof.iter = launched + j + 1;
                        if (graph)
                            GIAMG_HIP(hipGraphLaunch(H.it_exec, its));
                        else
                            iteration();
                    }
                    launched += todo;
                    GIAMG_HIP(hipMemcpyAsync(H.host_ctl, w.ctl, C_COUNT * sizeof(int),
                                             hipMemcpyDeviceToHost, its));
                    GIAMG_HIP(hipStreamSynchronize(its));
                    if (H.host_ctl[C_STOP] != 0 || launched >= H.opts.maxit) break;
                    chunk = 1;
                }
            }
            if (graph) {
                GIAMG_HIP(hipEventRecord(H.ev_join, its));
                GIAMG_HIP(hipStreamWaitEvent(s, H.ev_join, 0));
            }
            H.bytes = bytes0;
            const double part1 = H.it_part1, part2 = H.it_part2;
            launch_copy<double>(n, xi, x, s);
            iters = H.host_ctl[C_ITERS];
            const int stop = H.host_ctl[C_STOP];
            status = stop == 1 ? GIAMG_OK : stop == 2 ? GIAMG_EBREAKDOWN : GIAMG_ENOTCONV;
            H.last_iters = iters;
            prof_first = stop == 2 ? iters + 1 : iters;
            prof_second = stop == 1 ? iters - 1 : iters;
            // bytes of the work that ran: the iteration that stopped skipped its second half
            const int halves2 = std::max(0, (stop == 2 ? iters : iters - 1));
            H.bytes = bytes0 + 16.0 * n + part1 * (stop == 2 ? iters + 1 : iters) + part2 * halves2;
            fetch_scalars(H, w.scal);
            relres = std::sqrt(H.host_scal[S_RR]) / bnorm;
        } else if (!(relres < tol)) {
            status = GIAMG_ENOTCONV;
        }
    }
    GIAMG_HIP(hipEventRecord(H.ev1, s));
    const double bytes = H.bytes;
    if (H.prof.on != 0 || !H.prof.pending.empty()) {
        GIAMG_HIP(hipEventSynchronize(H.ev1));
        prof_harvest(H, iters, prof_first, prof_second);
    }
    // true residual at exit (outside the timed region)
    rinit(w.tmp, false);
    launch_reduce(gs, w.partial, gs, 2, w.scal + S_BB, s);
    fetch_scalars(H, w.scal);
    if (info) {
        float ms = 0.0f;
        GIAMG_HIP(hipEventElapsedTime(&ms, H.ev0, H.ev1));
        info->iters = iters;
        info->status = status;
        info->relres = relres;
        info->true_relres = bnorm > 0 ? std::sqrt(H.host_scal[S_RR]) / bnorm : 0.0;
        info->solve_ms = ms;
        info->bytes = bytes;
    }
    return status;
}

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex& scratch_mutex() {
    static std::mutex m;
    return m;
}
unsigned char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

size_t align256(size_t bytes) { return (bytes + 255) & ~size_t(255); }
}  // namespace

// Fixed per-device scratch of the allocation-free solve (giamg_solve_noalloc):
// the CG work vectors, block partials, scalars and control block of one
// solve at a time; every GPU holds its own copy until the process ends.  In
// host code `scratch` only names the symbol: its device address is looked
// up once per device, with that device current (noalloc_scratch_init, run by
// setup), and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

void noalloc_scratch_init() {
    int dev = 0;
    GIAMG_HIP(hipGetDevice(&dev));
    GIAMG_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, "device index beyond 63");
    std::lock_guard<std::mutex> lock(scratch_mutex());
    if (g_scratch_ptr[dev] != nullptr) return;
    void* ptr = nullptr;
    GIAMG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (ptr == nullptr) throw Error(GIAMG_EHIP, "no device address for the solve scratch");
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
}

int solve(Handle& H, const double* b, double* x, double tol, giamg_info* info) {
    CgWork w{H.x.get(), H.r.get(), H.z.get(), H.p.get(), H.q.get(), H.rold.get(), H.tmp.get(),
             H.partial.get(), H.scal.get(), H.ctl.get()};
    return solve_on(H, w, true, b, x, tol, info);
}

int solve_noalloc(Handle& H, int device, const double* b, double* x, double tol, giamg_info* info) {
    GIAMG_REQUIRE(device >= 0 && device < NOALLOC_MAX_DEVICES, "device index beyond 63");
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mutex());
        base = g_scratch_ptr[device];
    }
    if (base == nullptr) throw Error(GIAMG_EHIP, "solve scratch not set up on this device");
    const size_t vec = align256((size_t)std::max<int64_t>(H.n_nodes, 1) * sizeof(double));
    const size_t fixed = align256((size_t)H.partial_cap * sizeof(double)) +
                         align256(S_COUNT * sizeof(double)) + align256(C_COUNT * sizeof(int));
    const size_t need = 7 * vec + fixed;
    if (need > NOALLOC_SCRATCH_BYTES) {
        const size_t fit = (NOALLOC_SCRATCH_BYTES - std::min(fixed, NOALLOC_SCRATCH_BYTES)) /
                           (7 * sizeof(double));
        throw Error(GIAMG_EINVAL, "giamg_solve_noalloc: " + std::to_string(H.n_nodes) +
                                      " nodes need " + std::to_string(need) +
                                      " bytes of solve scratch, more than its fixed " +
                                      std::to_string(NOALLOC_SCRATCH_BYTES) + " (at most about " +
                                      std::to_string(fit) + " nodes with this hierarchy)");
    }
    unsigned char* c = base;
    auto take = [&](size_t bytes) {
        unsigned char* p = c;
        c += align256(bytes);
        return p;
    };
    CgWork w;
    w.x = reinterpret_cast<double*>(take(vec));
    w.r = reinterpret_cast<double*>(take(vec));
    w.z = reinterpret_cast<double*>(take(vec));
    w.p = reinterpret_cast<double*>(take(vec));
    w.q = reinterpret_cast<double*>(take(vec));
    w.rold = reinterpret_cast<double*>(take(vec));
    w.tmp = reinterpret_cast<double*>(take(vec));
    w.partial = reinterpret_cast<double*>(take((size_t)H.partial_cap * sizeof(double)));
    w.scal = reinterpret_cast<double*>(take(S_COUNT * sizeof(double)));
    w.ctl = reinterpret_cast<int*>(take(C_COUNT * sizeof(int)));
    const int prof = H.prof.on;   // profiling creates events: off for this call
    H.prof.on = 0;
    try {
        const int rc = solve_on(H, w, false, b, x, tol, info);
        H.prof.on = prof;
        return rc;
    } catch (...) {
        H.prof.on = prof;
        throw;
    }
}

// ---------------------------------------------------------------------------
// kernel timing in the solve's launch configuration
// ---------------------------------------------------------------------------
namespace {
template <typename T>
void time_kernel_t(Handle& H, int kernel, size_t l, int reps, double* ms, double* bytes) {
    Level& L = H.levels[l];
    const bool last = l + 1 == H.levels.size();
    GIAMG_REQUIRE(kernel == GIAMG_KERNEL_SPMV || !last, "no transfer or smoother on the coarsest level");
    SpmvArgs<T> a;
    int mode = SPMV_PLAIN;
    DevBuf<double> partial;
    if (kernel == GIAMG_KERNEL_CHEB_STEP || kernel == GIAMG_KERNEL_SPMV || kernel == GIAMG_KERNEL_CG_PRODUCT) {
        a = args_A<T>(L);
        a.v = LV<T>::d0(L); a.y = LV<T>::d1(L);
        if (kernel == GIAMG_KERNEL_CG_PRODUCT) {
            mode = SPMV_DOT;
            partial.alloc((size_t)std::max<int64_t>(a.nblk, 1));
            a.partial = partial.get();
        }
        if (kernel == GIAMG_KERNEL_CHEB_STEP) {
            const ChebCoef c = cheb_coef(H, L);
            mode = SPMV_CHEB_STEP;
            a.r = LV<T>::r(L); a.x = LV<T>::x(L);
            a.c1 = (T)(c.c1.empty() ? 0.0 : c.c1[0]);
            a.c2 = (T)(c.c2.empty() ? 0.0 : c.c2[0]);
            a.flags = 0;
        }
    } else if (kernel == GIAMG_KERNEL_RESTRICT) {
        Level& C = H.levels[l + 1];
        a = args_of<T>(L.R, LV<T>::R(L));
        a.v = LV<T>::t(L); a.y = LV<T>::f(C);
    } else if (kernel == GIAMG_KERNEL_PROLONG) {
        Level& C = H.levels[l + 1];
        mode = SPMV_ADD;
        a = args_of<T>(L.P, LV<T>::P(L));
        a.v = LV<T>::x(C); a.y = LV<T>::t(L);
    } else {
        throw Error(GIAMG_EINVAL, "unknown kernel");
    }
    // defined contents: zeros in every vector the kernel touches
    for (T* v : {LV<T>::d0(L), LV<T>::d1(L), LV<T>::r(L), LV<T>::x(L), LV<T>::t(L)})
        GIAMG_HIP(hipMemsetAsync(v, 0, L.n * sizeof(T), H.stream));
    if (!last) {
        Level& C = H.levels[l + 1];
        GIAMG_HIP(hipMemsetAsync(LV<T>::x(C), 0, C.n * sizeof(T), H.stream));
    }
    launch_spmv(mode, a, H.stream);   // warm-up
    // one event pair per launch, recorded by the dispatch itself at kernel
    // start and end: the average is the kernel's own duration
    std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
    double total = 0.0;
    try {
        for (auto& e : ev) GIAMG_HIP(hipEventCreate(&e));
        for (int i = 0; i < reps; ++i) {
            SpmvArgs<T> at = a;
            at.ev_start = ev[2 * i];
            at.ev_stop = ev[2 * i + 1];
            launch_spmv(mode, at, H.stream);
        }
        GIAMG_HIP(hipEventSynchronize(ev.back()));
        for (int i = 0; i < reps; ++i) {
            float t = 0.0f;
            GIAMG_HIP(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
            total += t;
        }
    } catch (...) {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        throw;
    }
    for (auto e : ev) (void)hipEventDestroy(e);
    *ms = total / reps;
    *bytes = spmv_bytes(mode, a);
}
}  // namespace

void profile_enable(Handle& H, int on) { H.prof.on = on; }

void profile_read(Handle& H, giamg_profile* out, bool reset) {
    *out = H.prof.acc;
    if (reset) H.prof.acc = giamg_profile{};
}

void time_kernel(Handle& H, int kernel, int level, int reps, double* ms, double* bytes) {
    AllocStreamScope alloc_scope(H.stream);
    GIAMG_REQUIRE(level >= 0 && level < (int)H.levels.size(), "level out of range");
    GIAMG_REQUIRE(reps >= 1 && reps <= 100000, "reps must be in [1, 100000]");
    if (kernel & GIAMG_OP_FP32) {
        GIAMG_REQUIRE(H.opts.precision == GIAMG_PREC_MIXED, "FP32 operators exist only in mixed mode");
        GIAMG_REQUIRE((kernel & ~GIAMG_OP_FP32) != GIAMG_KERNEL_CG_PRODUCT, "the CG product is FP64 only");
        time_kernel_t<float>(H, kernel & ~GIAMG_OP_FP32, level, reps, ms, bytes);
    } else {
        time_kernel_t<double>(H, kernel, level, reps, ms, bytes);
    }
}

// ---------------------------------------------------------------------------
// single steps for checking
// ---------------------------------------------------------------------------
namespace {
template <typename T>
void apply_t(Handle& H, int op, size_t l, const T* a, const T* b, T* out) {
    Level& L = H.levels[l];
    const bool last = l + 1 == H.levels.size();
    switch (op) {
        case GIAMG_OP_SPMV: {
            SpmvArgs<T> s = args_A<T>(L);
            s.v = a; s.y = out;
            run_spmv(H, SPMV_PLAIN, s);
            break;
        }
        case GIAMG_OP_RESIDUAL: residual<T>(H, L, a, b, out); break;
        case GIAMG_OP_RESTRICT:
            GIAMG_REQUIRE(!last, "no restriction on the coarsest level");
            restrict_to<T>(H, L, a, out);
            break;
        case GIAMG_OP_PROLONG_ADD:
            GIAMG_REQUIRE(!last, "no prolongation on the coarsest level");
            prolong_add<T>(H, L, a, out);
            break;
        case GIAMG_OP_PRESMOOTH:
            GIAMG_REQUIRE(!last, "no smoother on the coarsest level");
            smooth<T>(H, L, a, out, true);
            break;
        case GIAMG_OP_POSTSMOOTH:
            GIAMG_REQUIRE(!last, "no smoother on the coarsest level");
            smooth<T>(H, L, a, out, false);
            break;
        case GIAMG_OP_COARSE:
            GIAMG_REQUIRE(last, "direct solve only on the coarsest level");
            launch_coarse_apply<T>(H.nc, H.coarse_inv.get(), a, out, H.stream);
            break;
        case GIAMG_OP_VCYCLE: vcycle<T>(H, l, a, out); break;
        default: throw Error(GIAMG_EINVAL, "unknown operation");
    }
}
}  // namespace

void apply(Handle& H, int op, int level, const void* a, const void* b, void* out) {
    AllocStreamScope alloc_scope(H.stream);
    const int base = op & ~GIAMG_OP_FP32;
    if (H.opts.preconditioner != GIAMG_PRECOND_VCYCLE && base != GIAMG_OP_SPMV && base != GIAMG_OP_RESIDUAL)
        throw Error(GIAMG_ENOTSUP, "a Jacobi-preconditioned handle has no V-cycle steps");
    GIAMG_REQUIRE(level >= 0 && level < (int)H.levels.size(), "level out of range");
    GIAMG_REQUIRE(a != nullptr, "a is null");
    GIAMG_REQUIRE(b != nullptr || (op & ~GIAMG_OP_FP32) != GIAMG_OP_RESIDUAL,
                  "b is null (the residual needs x)");
    if (op & GIAMG_OP_FP32) {
        GIAMG_REQUIRE(H.opts.precision == GIAMG_PREC_MIXED, "FP32 operators exist only in mixed mode");
        apply_t<float>(H, op & ~GIAMG_OP_FP32, level, (const float*)a, (const float*)b, (float*)out);
    } else {
        apply_t<double>(H, op, level, (const double*)a, (const double*)b, (double*)out);
    }
    GIAMG_HIP(hipStreamSynchronize(H.stream));
}

}  // namespace giamg
