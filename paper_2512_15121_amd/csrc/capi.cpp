// extern "C" entry points of the GIAMG library: argument checks, error
// codes, the thread-local error message, and dispatch into the C++ core.
#include <cmath>
#include <cstring>
#include <string>

#include "internal.h"

struct giamg_s {
    giamg::Handle h;
    int device = 0;
};

struct giamg_hcsr_s {
    giamg::HostCSR m;
};

namespace giamg {
void build_hierarchy(Handle& H, const double* coords, const int32_t* l2g);
int solve(Handle& H, const double* b, double* x, double tol, giamg_info* info);
int solve_noalloc(Handle& H, int device, const double* b, double* x, double tol, giamg_info* info);
void profile_enable(Handle& H, int on);
void profile_read(Handle& H, giamg_profile* out, bool reset);
void read_bandwidth(int64_t bytes, int reps, double* gbs);
int solve_batch(Handle& H, const double* B, double* X, int32_t k, double tol, giamg_info* infos);
void apply(Handle& H, int op, int level, const void* a, const void* b, void* out);
void time_kernel(Handle& H, int kernel, int level, int reps, double* ms, double* bytes);
struct Session;
Session* session_create(Handle& H, int k, double tol);
void session_destroy(Session* S);
void session_admit(Session* S, const int* slot, const double* const* b, int count);
void session_step(Session* S, int iters);
void session_poll(Session* S, int* state, giamg_info* infos);
void session_retire(Session* S, int slot, double* x);
}  // namespace giamg

namespace giamg {
std::string& last_error() {
    thread_local std::string msg;
    return msg;
}

// ---- device memory (allocator registration) --------------------------------
namespace {
std::mutex& allocator_mutex() {
    static std::mutex m;
    return m;
}
Allocator& allocator_slot() {
    static Allocator a;
    return a;
}
thread_local hipStream_t t_alloc_stream = nullptr;
}  // namespace

Allocator registered_allocator() {
    std::lock_guard<std::mutex> lock(allocator_mutex());
    return allocator_slot();
}

hipStream_t alloc_stream() { return t_alloc_stream; }
AllocStreamScope::AllocStreamScope(hipStream_t s) : prev_(t_alloc_stream) { t_alloc_stream = s; }
AllocStreamScope::~AllocStreamScope() { t_alloc_stream = prev_; }

void* device_alloc(size_t bytes, Allocator& a, hipStream_t& s) {
    a = registered_allocator();
    s = t_alloc_stream;
    void* p = nullptr;
    if (a.alloc != nullptr) {
        p = a.alloc(bytes, reinterpret_cast<void*>(s), a.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p == nullptr)
        throw Error(GIAMG_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void device_release(void* p, const Allocator& a, hipStream_t s) {
    if (a.release != nullptr) {
        (void)hipStreamSynchronize(s);
        a.release(p, a.ctx);
    } else {
        (void)hipFree(p);
    }
}
}  // namespace giamg

namespace giamg {
void check_setup_args(const double* coords, int64_t n_nodes, const int32_t* l2g, int64_t n_elem,
                      int32_t p, double lambda, const giamg_opts& o) {
    GIAMG_REQUIRE(coords != nullptr && l2g != nullptr, "coords and l2g must be non-null");
    GIAMG_REQUIRE(n_nodes > 0 && n_elem > 0, "n_nodes and n_elem must be positive");
    GIAMG_REQUIRE(n_nodes < (int64_t(1) << 31) - 1, "n_nodes exceeds the int32 index range");
    GIAMG_REQUIRE(p >= 1 && p <= 10, "order p must be in [1, 10]");
    GIAMG_REQUIRE(std::isfinite(lambda) && lambda >= 0.0, "lambda must be finite and >= 0");
    GIAMG_REQUIRE(o.smoother == GIAMG_SMOOTHER_CHEBYSHEV || o.smoother == GIAMG_SMOOTHER_JACOBI,
                  "unknown smoother");
    GIAMG_REQUIRE(o.degree >= 1 && o.degree <= 16, "degree must be in [1, 16]");
    GIAMG_REQUIRE(o.omega > 0.0 && o.omega < 2.0, "omega must be in (0, 2)");
    GIAMG_REQUIRE(o.coarse_max >= 1 && o.max_levels >= 1 && o.max_levels <= 32,
                  "bad coarse_max / max_levels");
    GIAMG_REQUIRE(o.bc == GIAMG_BC_DIRICHLET || o.bc == GIAMG_BC_PIN, "unknown bc");
    GIAMG_REQUIRE(o.bc != GIAMG_BC_PIN || (o.pin_node >= 0 && o.pin_node < n_nodes),
                  "pin_node out of range");
    GIAMG_REQUIRE(o.precision == GIAMG_PREC_FP64 || o.precision == GIAMG_PREC_MIXED,
                  "unknown precision");
    GIAMG_REQUIRE(o.maxit >= 0, "maxit must be >= 0");
    GIAMG_REQUIRE(o.power_iters >= 1, "power_iters must be >= 1");
    GIAMG_REQUIRE(o.cheb_lo > 0.0 && o.cheb_hi > o.cheb_lo, "need 0 < cheb_lo < cheb_hi");
    GIAMG_REQUIRE(o.direct_gathers == 0 || o.direct_gathers == 1, "direct_gathers must be 0 or 1");
    GIAMG_REQUIRE(o.graph_launch == 0 || o.graph_launch == 1, "graph_launch must be 0 or 1");
    GIAMG_REQUIRE(o.basis == GIAMG_BASIS_NODAL || o.basis == GIAMG_BASIS_MODAL, "unknown basis");
    GIAMG_REQUIRE(o.batch_kernel >= GIAMG_BATCH_AUTO && o.batch_kernel <= GIAMG_BATCH_GROUP,
                  "unknown batch_kernel");
    GIAMG_REQUIRE(o.row_groups == 0 || o.row_groups == 1, "row_groups must be 0 or 1");
    GIAMG_REQUIRE(o.lean_max_nnz >= 0, "lean_max_nnz must be >= 0");
    GIAMG_REQUIRE(o.keep_boundary == 0 || o.keep_boundary == 1, "keep_boundary must be 0 or 1");
    GIAMG_REQUIRE(o.theta >= 0.0 && o.theta <= 1.0, "theta must be in [0, 1]");
    GIAMG_REQUIRE(o.preconditioner == GIAMG_PRECOND_VCYCLE || o.preconditioner == GIAMG_PRECOND_JACOBI,
                  "unknown preconditioner");
    GIAMG_REQUIRE(o.preconditioner == GIAMG_PRECOND_VCYCLE || o.precision == GIAMG_PREC_FP64,
                  "the Jacobi preconditioner runs in FP64 only (precision must be FP64)");
    GIAMG_REQUIRE(o.assembly == GIAMG_ASSEMBLY_AUTO || o.assembly == GIAMG_ASSEMBLY_DEVICE ||
                      o.assembly == GIAMG_ASSEMBLY_HOST,
                  "unknown assembly mode");
    {
        int prev = p;
        for (int i = 0; i < 8 && o.schedule[i] != 0; ++i) {
            GIAMG_REQUIRE(o.schedule[i] >= 1 && o.schedule[i] < prev,
                          "schedule must decrease from p and stay >= 1");
            prev = o.schedule[i];
        }
    }
    const int64_t nl = (int64_t)(p + 1) * (p + 1) * (p + 1);
    for (int64_t i = 0; i < n_elem * nl; ++i)
        GIAMG_REQUIRE(l2g[i] >= 0 && l2g[i] < n_nodes, "l2g entry out of range");
    for (int64_t e = 0; e < n_elem; ++e) {
        const int32_t* g = l2g + e * nl;
        for (int c = 0; c < 8; ++c) {
            int i = ((c >> 2) & 1) * p, j = ((c >> 1) & 1) * p, k = (c & 1) * p;
            const double* x = coords + (int64_t)g[((p + 1) * i + j) * (p + 1) + k] * 3;
            GIAMG_REQUIRE(std::isfinite(x[0]) && std::isfinite(x[1]) && std::isfinite(x[2]),
                          "non-finite corner coordinate");
        }
    }
}
}  // namespace giamg

namespace {
#define g_last_error (::giamg::last_error())

template <typename F>
int guarded(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const giamg::Error& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return GIAMG_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return GIAMG_EINVAL;
    }
}

int bind_device(giamg_s* h) {
    if (!h) throw giamg::Error(GIAMG_EINVAL, "null handle");
    GIAMG_HIP(hipSetDevice(h->device));
    return 0;
}
}  // namespace

extern "C" {

int giamg_set_allocator(giamg_alloc_fn alloc, giamg_release_fn release, void* ctx) {
    if ((alloc == nullptr) != (release == nullptr)) {
        giamg::last_error() = "alloc and release must both be set or both be NULL";
        return GIAMG_EINVAL;
    }
    std::lock_guard<std::mutex> lock(giamg::allocator_mutex());
    giamg::allocator_slot() = giamg::Allocator{alloc, release, alloc ? ctx : nullptr};
    return GIAMG_OK;
}

void giamg_default_opts(giamg_opts* o) {
    if (!o) return;
    o->smoother = GIAMG_SMOOTHER_CHEBYSHEV;
    o->degree = 2;
    o->omega = 2.0 / 3.0;
    o->coarse_max = 2000;
    o->max_levels = 10;
    o->bc = GIAMG_BC_DIRICHLET;
    o->pin_node = 0;
    o->precision = GIAMG_PREC_FP64;
    o->maxit = 500;
    o->agg_seed = 0;
    o->power_iters = 20;
    o->cheb_lo = 0.1;
    o->cheb_hi = 1.1;
    o->direct_gathers = 0;
    o->graph_launch = 0;
    o->basis = GIAMG_BASIS_NODAL;
    for (int i = 0; i < 8; ++i) o->schedule[i] = 0;
    o->batch_kernel = GIAMG_BATCH_AUTO;
    o->row_groups = 0;
    o->pad = 0;
    o->lean_max_nnz = 2000000;
    o->keep_boundary = 0;
    o->pad2 = 0;
    o->theta = 0.0;
    o->preconditioner = GIAMG_PRECOND_VCYCLE;
    o->assembly = GIAMG_ASSEMBLY_AUTO;
}

int giamg_setup(const double* coords, int64_t n_nodes, const int32_t* l2g, int64_t n_elem,
                int32_t p, double lambda, const giamg_opts* opts, void* stream,
                giamg_handle* out) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(out != nullptr, "out is null");
        giamg_opts o;
        giamg_default_opts(&o);
        if (opts) o = *opts;
        giamg::check_setup_args(coords, n_nodes, l2g, n_elem, p, lambda, o);
        auto* h = new giamg_s();
        try {
            GIAMG_HIP(hipGetDevice(&h->device));
            h->h.stream = reinterpret_cast<hipStream_t>(stream);
            h->h.opts = o;
            h->h.porder = p;
            h->h.lambda = lambda;
            h->h.n_nodes = n_nodes;
            h->h.n_elem = n_elem;
            giamg::build_hierarchy(h->h, coords, l2g);
        } catch (...) {
            (void)hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
            delete h;
            throw;
        }
        *out = h;
        return GIAMG_OK;
    });
}

void giamg_free(giamg_handle h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->h.stream);
    delete h;
}

int giamg_solve(giamg_handle h, const double* b, double* x, double tol, giamg_info* info) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(b != nullptr && x != nullptr, "b and x must be non-null");
        GIAMG_REQUIRE(tol >= 0.0 && std::isfinite(tol), "tol must be finite and >= 0");
        const int rc = giamg::solve(h->h, b, x, tol, info);
        if (rc == GIAMG_EBREAKDOWN) g_last_error = "CG breakdown (p^T A p <= 0 or non-finite)";
        if (rc == GIAMG_ENOTCONV) g_last_error = "iteration cap reached";
        return rc;
    });
}

int giamg_solve_noalloc(giamg_handle h, const double* b, double* x, double tol, giamg_info* info) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(b != nullptr && x != nullptr, "b and x must be non-null");
        GIAMG_REQUIRE(tol >= 0.0 && std::isfinite(tol), "tol must be finite and >= 0");
        const int rc = giamg::solve_noalloc(h->h, h->device, b, x, tol, info);
        if (rc == GIAMG_EBREAKDOWN) g_last_error = "CG breakdown (p^T A p <= 0 or non-finite)";
        if (rc == GIAMG_ENOTCONV) g_last_error = "iteration cap reached";
        return rc;
    });
}

int giamg_solve_batch(giamg_handle h, const double* B, double* X, int32_t k, double tol,
                      giamg_info* infos) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(B != nullptr && X != nullptr, "B and X must be non-null");
        GIAMG_REQUIRE(k >= 1, "k must be >= 1");
        GIAMG_REQUIRE(tol >= 0.0 && std::isfinite(tol), "tol must be finite and >= 0");
        if (h->h.opts.preconditioner != GIAMG_PRECOND_VCYCLE)
            throw giamg::Error(GIAMG_ENOTSUP, "batched solves need the V-cycle preconditioner");
        return giamg::solve_batch(h->h, B, X, k, tol, infos);
    });
}

int giamg_hierarchy_info(giamg_handle h, int32_t* n_levels, int64_t* rows, int64_t* nnz,
                         int32_t cap) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(h != nullptr && n_levels != nullptr, "null handle or n_levels");
        GIAMG_REQUIRE(cap >= 0, "cap must be >= 0");
        GIAMG_REQUIRE(cap == 0 || (rows != nullptr && nnz != nullptr),
                      "rows and nnz must be non-null when cap > 0");
        const auto& lv = h->h.levels;
        *n_levels = (int32_t)lv.size();
        for (int32_t l = 0; l < cap && l < (int32_t)lv.size(); ++l) {
            rows[l] = lv[l].n;
            nnz[l] = lv[l].A.nnz;
        }
        return GIAMG_OK;
    });
}

int giamg_num_levels(giamg_handle h) {
    return guarded([&]() -> int {
        bind_device(h);
        return (int)h->h.levels.size();
    });
}

int giamg_level_describe(giamg_handle h, int32_t level, giamg_level_desc* out) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(out != nullptr, "out is null");
        GIAMG_REQUIRE(level >= 0 && level < (int)h->h.levels.size(), "level out of range");
        const giamg::Level& L = h->h.levels[level];
        out->kind = L.kind;
        out->order = L.order;
        out->coarsest = level + 1 == (int)h->h.levels.size();
        out->device_assembly = L.device_assembled ? 1 : 0;
        out->rows = L.n;
        out->nnz_A = L.A.nnz;
        out->nnz_P = L.P.nnz;
        out->nnz_R = L.R.nnz;
        out->lam_hat = L.lam_hat;
        out->nnz_AP = L.AP.nnz;
        out->staged_nnz_A = L.A.blk.nnz_staged;
        out->runs_A = L.A.blk.nruns;
        out->groups_A = L.A.gnblk > 0 ? L.A.ggroups : 0;
        out->group_entries_A = L.A.gnblk > 0 ? L.A.gentries : 0;
        out->lean_A = L.A.lean ? 1 : 0;
        return GIAMG_OK;
    });
}

int giamg_level_csr(giamg_handle h, int32_t level, int32_t which, int64_t* row_ptr, int32_t* col,
                    double* val) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(level >= 0 && level < (int)h->h.levels.size(), "level out of range");
        const giamg::Level& L = h->h.levels[level];
        const giamg::DevCSR* M = which == GIAMG_MAT_A ? &L.A
                                 : which == GIAMG_MAT_P ? &L.P
                                 : which == GIAMG_MAT_R ? &L.R
                                 : which == GIAMG_MAT_AP ? &L.AP
                                                         : nullptr;
        GIAMG_REQUIRE(M != nullptr, "unknown matrix");
        GIAMG_REQUIRE(M->nrows > 0 || which == GIAMG_MAT_A, "matrix absent on this level");
        hipStream_t s = h->h.stream;
        if (row_ptr)
            GIAMG_HIP(hipMemcpyAsync(row_ptr, M->rp.get(), (M->nrows + 1) * sizeof(int64_t),
                                     hipMemcpyDeviceToHost, s));
        if (col && M->nnz)
            GIAMG_HIP(hipMemcpyAsync(col, M->ci.get(), M->nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (val && M->nnz)
            GIAMG_HIP(hipMemcpyAsync(val, M->val.get(), M->nnz * sizeof(double), hipMemcpyDeviceToHost, s));
        GIAMG_HIP(hipStreamSynchronize(s));
        return GIAMG_OK;
    });
}

int giamg_level_l2g(giamg_handle h, int32_t level, int32_t* out) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(out != nullptr, "out is null");
        GIAMG_REQUIRE(level >= 0 && level < (int)h->h.levels.size(), "level out of range");
        const giamg::Level& L = h->h.levels[level];
        GIAMG_REQUIRE(L.kind == GIAMG_LEVEL_P, "not a p-level");
        std::memcpy(out, L.l2g.data(), L.l2g.size() * sizeof(int32_t));
        return GIAMG_OK;
    });
}

int giamg_level_aggregates(giamg_handle h, int32_t level, int32_t* out) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(out != nullptr, "out is null");
        GIAMG_REQUIRE(level >= 0 && level < (int)h->h.levels.size(), "level out of range");
        const giamg::Level& L = h->h.levels[level];
        GIAMG_REQUIRE(!L.agg.empty(), "the next level is not an aggregation level");
        std::memcpy(out, L.agg.data(), L.agg.size() * sizeof(int32_t));
        return GIAMG_OK;
    });
}

int giamg_constrained(giamg_handle h, uint8_t* mask) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(mask != nullptr, "mask is null");
        std::memcpy(mask, h->h.constrained.data(), h->h.constrained.size());
        return GIAMG_OK;
    });
}

int giamg_apply(giamg_handle h, int32_t op, int32_t level, const void* a, const void* b, void* out) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(out != nullptr, "out is null");
        giamg::apply(h->h, op, level, a, b, out);
        return GIAMG_OK;
    });
}

int giamg_quadrature_points(giamg_handle h, double* xq) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(xq != nullptr, "xq is null");
        giamg::quadrature_points(h->h.corners, h->h.n_elem, h->h.porder, xq);
        return GIAMG_OK;
    });
}

int giamg_load_vector(giamg_handle h, const double* fq, double* b) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(fq != nullptr && b != nullptr, "fq and b must be non-null");
        giamg::load_vector(h->h.corners, h->h.l2g.data(), h->h.n_elem, h->h.porder, h->h.n_nodes,
                           h->h.constrained, fq, b, h->h.opts.basis);
        return GIAMG_OK;
    });
}

int giamg_setup_times(giamg_handle h, double* ms) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(ms != nullptr, "ms is null");
        for (int i = 0; i < 7; ++i) ms[i] = h->h.setup_ms[i];
        return GIAMG_OK;
    });
}

int giamg_hcsr_size(giamg_hcsr m, int64_t* rows, int64_t* cols, int64_t* nnz) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(m != nullptr, "null matrix");
        if (rows) *rows = m->m.nrows;
        if (cols) *cols = m->m.ncols;
        if (nnz) *nnz = m->m.nnz();
        return GIAMG_OK;
    });
}

int giamg_hcsr_copy(giamg_hcsr m, int64_t* row_ptr, int32_t* col, double* val) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(m != nullptr, "null matrix");
        if (row_ptr) std::memcpy(row_ptr, m->m.rp.data(), m->m.rp.size() * sizeof(int64_t));
        if (col) std::memcpy(col, m->m.ci.data(), m->m.ci.size() * sizeof(int32_t));
        if (val) std::memcpy(val, m->m.val.data(), m->m.val.size() * sizeof(double));
        return GIAMG_OK;
    });
}

void giamg_hcsr_free(giamg_hcsr m) { delete m; }

int giamg_host_boundary(const int32_t* l2g, int64_t n_elem, int32_t p, int64_t n_nodes,
                        int32_t basis, uint8_t* mask) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(l2g && mask && n_elem > 0 && n_nodes > 0 && p >= 1 && p <= 10, "bad arguments");
        GIAMG_REQUIRE(basis == GIAMG_BASIS_NODAL || basis == GIAMG_BASIS_MODAL, "unknown basis");
        const int64_t nl = (int64_t)(p + 1) * (p + 1) * (p + 1);
        for (int64_t i = 0; i < n_elem * nl; ++i)
            GIAMG_REQUIRE(l2g[i] >= 0 && l2g[i] < n_nodes, "l2g entry out of range");
        auto m = giamg::boundary_mask(l2g, n_elem, p, n_nodes, basis);
        std::memcpy(mask, m.data(), m.size());
        return GIAMG_OK;
    });
}

int giamg_host_assemble(const double* coords, int64_t n_nodes, const int32_t* l2g,
                        int64_t n_elem, int32_t p, double lambda, int32_t bc, int64_t pin_node,
                        int32_t basis, giamg_hcsr* A_out) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(coords && l2g && A_out && n_elem > 0 && n_nodes > 0 && p >= 1 && p <= 10,
                      "bad arguments");
        GIAMG_REQUIRE(basis == GIAMG_BASIS_NODAL || basis == GIAMG_BASIS_MODAL, "unknown basis");
        GIAMG_REQUIRE(bc == GIAMG_BC_DIRICHLET || (bc == GIAMG_BC_PIN && pin_node >= 0 &&
                                                   pin_node < n_nodes), "bad boundary condition");
        const int64_t nl = (int64_t)(p + 1) * (p + 1) * (p + 1);
        for (int64_t i = 0; i < n_elem * nl; ++i)
            GIAMG_REQUIRE(l2g[i] >= 0 && l2g[i] < n_nodes, "l2g entry out of range");
        std::vector<uint8_t> cons;
        if (bc == GIAMG_BC_DIRICHLET) {
            cons = giamg::boundary_mask(l2g, n_elem, p, n_nodes, basis);
        } else {
            cons.assign(n_nodes, 0);
            cons[pin_node] = 1;
        }
        std::vector<double> corners;
        giamg::element_corners(coords, l2g, n_elem, p, corners, basis);
        giamg::HostCSR A = giamg::assemble_fine(corners, l2g, n_elem, p, n_nodes, lambda, cons, basis);
        *A_out = new giamg_hcsr_s{std::move(A)};
        return GIAMG_OK;
    });
}

int giamg_host_p_transfer(const int32_t* l2g, int64_t n_elem, int32_t p, int32_t q,
                          int64_t n_fine, const uint8_t* free_mask, int32_t basis,
                          int32_t* l2g_next, int64_t* n_coarse, giamg_hcsr* P_out) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(l2g && free_mask && l2g_next && n_coarse && P_out, "null argument");
        GIAMG_REQUIRE(basis == GIAMG_BASIS_NODAL || basis == GIAMG_BASIS_MODAL, "unknown basis");
        GIAMG_REQUIRE(p <= 10 && q >= 1 && q < p, "need 1 <= q < p <= 10");
        GIAMG_REQUIRE(n_elem > 0 && n_fine > 0, "n_elem and n_fine must be positive");
        const int64_t nl = (int64_t)(p + 1) * (p + 1) * (p + 1);
        std::vector<int32_t> g(l2g, l2g + n_elem * nl);
        for (auto v : g) GIAMG_REQUIRE(v >= -1 && v < n_fine, "l2g entry out of range");
        std::vector<uint8_t> fm(free_mask, free_mask + n_fine);
        std::vector<int32_t> nx;
        giamg::HostCSR P = giamg::p_transfer(g, n_elem, p, q, n_fine, fm, nx, *n_coarse, basis);
        std::memcpy(l2g_next, nx.data(), nx.size() * sizeof(int32_t));
        *P_out = new giamg_hcsr_s{std::move(P)};
        return GIAMG_OK;
    });
}

int giamg_host_aggregate(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t n,
                         uint64_t seed, double theta, int32_t* agg, int64_t* n_agg,
                         giamg_hcsr* P_out) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(row_ptr && col && val && agg && n_agg && P_out && n > 0, "null argument");
        GIAMG_REQUIRE(theta >= 0.0 && theta <= 1.0, "theta must be in [0, 1]");
        GIAMG_REQUIRE(n < (int64_t(1) << 31) - 1, "n exceeds the int32 index range");
        GIAMG_REQUIRE(row_ptr[0] == 0, "row_ptr[0] must be 0");
        for (int64_t i = 0; i < n; ++i)
            GIAMG_REQUIRE(row_ptr[i + 1] >= row_ptr[i], "row_ptr must be non-decreasing");
        giamg::HostCSR A;
        A.nrows = A.ncols = n;
        A.rp.assign(row_ptr, row_ptr + n + 1);
        A.ci.assign(col, col + A.rp.back());
        A.val.assign(val, val + A.rp.back());
        for (auto c : A.ci) GIAMG_REQUIRE(c >= 0 && c < n, "column out of range");
        std::vector<int32_t> a;
        giamg::HostCSR P = giamg::sa_transfer(A, seed, theta, a, *n_agg);
        std::memcpy(agg, a.data(), a.size() * sizeof(int32_t));
        *P_out = new giamg_hcsr_s{std::move(P)};
        return GIAMG_OK;
    });
}

int giamg_host_coarse_inverse(const double* A, int64_t n, double* inv) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(A != nullptr && inv != nullptr, "null argument");
        GIAMG_REQUIRE(n >= 1 && n <= 16384, "n must be in [1, 16384]");
        std::vector<double> a(A, A + n * n), out;
        GIAMG_REQUIRE(giamg::spd_inverse(a, n, out), "matrix is not positive definite");
        std::memcpy(inv, out.data(), out.size() * sizeof(double));
        return GIAMG_OK;
    });
}

int giamg_time_kernel(giamg_handle h, int32_t kernel, int32_t level, int32_t reps, double* ms,
                      double* bytes) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(ms != nullptr && bytes != nullptr, "null output");
        giamg::time_kernel(h->h, kernel, level, reps, ms, bytes);
        return GIAMG_OK;
    });
}

struct giamg_session_s {
    giamg::Session* s = nullptr;
    giamg_s* owner = nullptr;
};

int giamg_session_create(giamg_handle h, int32_t slots, double tol, giamg_session* out) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(out != nullptr, "out is null");
        GIAMG_REQUIRE(tol >= 0.0 && std::isfinite(tol), "tol must be finite and >= 0");
        if (h->h.opts.preconditioner != GIAMG_PRECOND_VCYCLE)
            throw giamg::Error(GIAMG_ENOTSUP, "sessions need the V-cycle preconditioner");
        giamg::Session* S = giamg::session_create(h->h, slots, tol);
        try {
            *out = new giamg_session_s{S, h};
        } catch (...) {
            giamg::session_destroy(S);
            throw;
        }
        return GIAMG_OK;
    });
}

int giamg_session_admit(giamg_session s, int32_t count, const int32_t* slots, const double* const* b) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(s && slots && b, "null argument");
        bind_device(s->owner);
        for (int i = 0; i < count; ++i) GIAMG_REQUIRE(b[i] != nullptr, "null right-hand side");
        giamg::session_admit(s->s, slots, b, count);
        return GIAMG_OK;
    });
}

int giamg_session_step(giamg_session s, int32_t iters) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(s && iters >= 0, "bad argument");
        bind_device(s->owner);
        giamg::session_step(s->s, iters);
        return GIAMG_OK;
    });
}

int giamg_session_poll(giamg_session s, int32_t* running, giamg_info* infos) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(s && running, "null argument");
        bind_device(s->owner);
        giamg::session_poll(s->s, running, infos);
        return GIAMG_OK;
    });
}

int giamg_session_retire(giamg_session s, int32_t slot, double* x) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(s && x, "null argument");
        bind_device(s->owner);
        giamg::session_retire(s->s, slot, x);
        return GIAMG_OK;
    });
}

void giamg_session_free(giamg_session s) {
    if (!s) return;
    (void)hipSetDevice(s->owner->device);
    giamg::session_destroy(s->s);
    delete s;
}

int giamg_profile_enable(giamg_handle h, int32_t on) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(on >= 0 && on <= 2, "on must be 0, 1 or 2");
        giamg::profile_enable(h->h, on);
        return GIAMG_OK;
    });
}

int giamg_profile_read(giamg_handle h, giamg_profile* out, int32_t reset) {
    return guarded([&]() -> int {
        bind_device(h);
        GIAMG_REQUIRE(out != nullptr, "out is null");
        GIAMG_REQUIRE(reset == 0 || reset == 1, "reset must be 0 or 1");
        giamg::profile_read(h->h, out, reset != 0);
        return GIAMG_OK;
    });
}

int giamg_read_bandwidth(int64_t bytes, int32_t reps, double* gbs) {
    return guarded([&]() -> int {
        GIAMG_REQUIRE(gbs != nullptr, "gbs is null");
        giamg::read_bandwidth(bytes, reps, gbs);
        return GIAMG_OK;
    });
}

const char* giamg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
