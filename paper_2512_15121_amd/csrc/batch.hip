// Batched solves: k right-hand sides against one hierarchy.
//
// Block vectors are row-major [n][k]: the entry of right-hand side j at row i
// sits at i*k + j, so one nonzero a_ic multiplies a contiguous run X[c][0:k]
// and every CSR entry read from HBM is reused k times.  The V-cycle
// (Algorithm 1) runs as block sparse-times-dense products (SpMM); each column
// keeps its own CG scalars and stops on its own (masked updates).  All
// per-column decisions happen on the device, so one CG iteration is captured
// once in a hipGraph and replayed; the host reads the number of active
// columns after each chunk of replays.
//
// Reproducibility: the value of column j depends only on column j's data,
// never on k or on the tile shape the tuner picks: row sums run over the
// nonzeros in CSR order and the column dot products use a fixed row
// partition.  A right-hand side gives the same bits alone or in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <memory>

#include "kernels.h"

namespace giamg {

namespace {

constexpr int BW = 64;              // wavefront width
constexpr int DOT_ROWS = 256;       // rows per column-dot block (fixed)
constexpr int MAX_K = 1024;
constexpr int CHUNK = 4;            // graph replays between host checks
constexpr int GROUP_MAX = 8;        // rows per row group of the group kernel

template <typename T>
struct SpmmArgs {
    const int64_t* rp = nullptr;
    const int32_t* ci = nullptr;
    const T* val = nullptr;
    int64_t n = 0;
    int k = 1;
    const T* v = nullptr;      // gathered block [ncols][k]
    T* y = nullptr;
    const T* f = nullptr;
    const T* dinv = nullptr;   // per row
    T* r = nullptr;
    T* x = nullptr;
    T c1 = 0, c2 = 0, inv_theta = 0, omega = 0;
    int flags = 0;
    const int* run = nullptr;  // skip all work when *run == 0
    const int32_t* gptr = nullptr;   // row groups (spmm_group_kernel only)
    const int32_t* grows = nullptr;
    int64_t ngroups = 0;
};

// Row-local tail of a block product: acc = (A v)[row][col].
template <typename T, int MODE>
__device__ __forceinline__ void spmm_epilogue(const SpmmArgs<T>& a, int64_t row, int64_t col, T acc) {
    const int64_t idx = row * a.k + col;
    if constexpr (MODE == SPMV_PLAIN) {
        a.y[idx] = acc;
    } else if constexpr (MODE == SPMV_RESID) {
        a.y[idx] = a.f[idx] - acc;
    } else if constexpr (MODE == SPMV_ADD) {
        a.y[idx] += acc;
    } else if constexpr (MODE == SPMV_CHEB_INIT) {
        const T res = a.dinv[row] * (a.f[idx] - acc);
        a.r[idx] = res;
        a.y[idx] = res * a.inv_theta;
    } else if constexpr (MODE == SPMV_CHEB_STEP) {
        const T rr = a.r[idx] - a.dinv[row] * acc;
        const T dold = a.v[idx];
        const T dn = a.c1 * dold + a.c2 * rr;
        a.r[idx] = rr;
        a.y[idx] = dn;
        const T inc = (a.flags & CHEB_LAST) ? dold + dn : dold;
        a.x[idx] = ((a.flags & CHEB_ASSIGN) ? T(0) : a.x[idx]) + inc;
    } else if constexpr (MODE == SPMV_JACOBI) {
        a.y[idx] = a.v[idx] + a.omega * a.dinv[row] * (a.f[idx] - acc);
    }
}

// One wavefront covers RPW = 64 / KT rows; KT lanes per row take KT columns.
template <typename T, int MODE, int KT, int WPB>
__global__ void __launch_bounds__(WPB* BW) spmm_kernel(SpmmArgs<T> a) {
    if (a.run && *a.run == 0) return;
    constexpr int RPW = BW / KT;
    const int lane = threadIdx.x % BW, wave = threadIdx.x / BW;
    const int sub = lane / KT, cl = lane % KT;
    const int64_t row = ((int64_t)blockIdx.x * WPB + wave) * RPW + sub;
    const int64_t col = (int64_t)blockIdx.y * KT + cl;
    if (row >= a.n || col >= a.k) return;
    const int64_t k = a.k;
    const int64_t s = a.rp[row], e = a.rp[row + 1];
    T acc = 0;
    int64_t j = s;
    for (; j + 3 < e; j += 4) {
        const int32_t c0 = a.ci[j], c1 = a.ci[j + 1], c2 = a.ci[j + 2], c3 = a.ci[j + 3];
        const T a0 = a.val[j], a1 = a.val[j + 1], a2 = a.val[j + 2], a3 = a.val[j + 3];
        const T x0 = a.v[c0 * k + col], x1 = a.v[c1 * k + col];
        const T x2 = a.v[c2 * k + col], x3 = a.v[c3 * k + col];
        acc += a0 * x0;
        acc += a1 * x1;
        acc += a2 * x2;
        acc += a3 * x3;
    }
    for (; j < e; ++j) acc += a.val[j] * a.v[a.ci[j] * k + col];
    spmm_epilogue<T, MODE>(a, row, col, acc);
}

__device__ __forceinline__ float lane_value(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_value(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One wavefront per row, 64 columns per wave (blockIdx.y selects the column
// tile).  The lanes fetch 64 consecutive (column, value) pairs of the row in
// one coalesced access each and hand them to the whole wave by readlane, so
// each gather of a block-vector row v[c][tile] is one load with a
// wave-uniform base instead of three per-lane loads.  The row sum runs over
// the nonzeros in CSR order, as in spmm_kernel, so both give the same bits.
// Lanes past k read column k-1 (in bounds) and store nothing.
template <typename T, int MODE, int WPB>
__global__ void __launch_bounds__(WPB* BW) spmm_wave_kernel(SpmmArgs<T> a) {
    if (a.run && *a.run == 0) return;
    constexpr int U = 8;   // gathers in flight per wave
    const int lane = threadIdx.x % BW;
    const int64_t row = (int64_t)blockIdx.x * WPB + threadIdx.x / BW;
    if (row >= a.n) return;
    const int64_t k = a.k;
    const int64_t col = (int64_t)blockIdx.y * BW + lane;
    const int64_t lc = col < k ? col : k - 1;
    const int64_t s = a.rp[row], e = a.rp[row + 1];
    T acc = 0;
    for (int64_t b = s; b < e; b += BW) {
        const int m = (int)min((int64_t)BW, e - b);
        const int li = lane < m ? lane : m - 1;
        const int32_t cw = a.ci[b + li];
        const T aw = a.val[b + li];
        int t = 0;
        for (; t + U <= m; t += U) {
            T xs[U], as[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t c = __builtin_amdgcn_readlane(cw, t + u);
                as[u] = lane_value(aw, t + u);
                xs[u] = a.v[c * k + lc];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += as[u] * xs[u];
        }
        for (; t < m; ++t) {
            const int64_t c = __builtin_amdgcn_readlane(cw, t);
            acc += lane_value(aw, t) * a.v[c * k + lc];
        }
    }
    if (col < k) spmm_epilogue<T, MODE>(a, row, col, acc);
}

// The G rows of one group share their column list; the wave reads each
// block-vector row v[c][tile] once and applies it to all G rows.  Row i of
// the group sums over its nonzeros in CSR order, as in spmm_kernel.  FP64
// form: each lane loads one value per row of a 64-entry chunk and the wave
// hands them out by readlane.
template <typename T, int MODE, int G>
__device__ __forceinline__ void group_rows_readlane(const SpmmArgs<T>& a, int32_t row_lane, int64_t start_lane,
                                           int lane, int64_t col, int64_t lc) {
    constexpr int U = G >= 4 ? 4 : 8;   // gathers in flight per wave
    const int64_t k = a.k;
    int64_t r[G], st[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
        r[i] = __builtin_amdgcn_readlane(row_lane, i);
        const int lo = __builtin_amdgcn_readlane((int)start_lane, i);
        const int hi = __builtin_amdgcn_readlane((int)(start_lane >> 32), i);
        st[i] = ((int64_t)hi << 32) | (uint32_t)lo;
    }
    const int64_t m = a.rp[r[0] + 1] - st[0];
    T acc[G];
#pragma unroll
    for (int i = 0; i < G; ++i) acc[i] = 0;
    for (int64_t b = 0; b < m; b += BW) {
        const int mb = (int)min((int64_t)BW, m - b);
        const int li = lane < mb ? lane : mb - 1;
        const int32_t cw = a.ci[st[0] + b + li];
        T vw[G];
#pragma unroll
        for (int i = 0; i < G; ++i) vw[i] = a.val[st[i] + b + li];
        int t = 0;
        for (; t + U <= mb; t += U) {
            T xs[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t c = __builtin_amdgcn_readlane(cw, t + u);
                xs[u] = a.v[c * k + lc];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int i = 0; i < G; ++i) acc[i] += lane_value(vw[i], t + u) * xs[u];
        }
        for (; t < mb; ++t) {
            const int64_t c = __builtin_amdgcn_readlane(cw, t);
            const T x = a.v[c * k + lc];
#pragma unroll
            for (int i = 0; i < G; ++i) acc[i] += lane_value(vw[i], t) * x;
        }
    }
    if (col < k) {
#pragma unroll
        for (int i = 0; i < G; ++i) spmm_epilogue<T, MODE>(a, r[i], col, acc[i]);
    }
}

// FP32 form of the same: the rows' values come in chunks of 64 per row by
// coalesced loads into the wave's LDS area wv ([GROUP_MAX][64]) and enter the
// multiply-adds by uniform-address (broadcast) LDS reads, four values per
// read, instead of one readlane per value (FP32 Chebyshev step 209 -> 185 us,
// residual 186 -> 157 us at 20^3 p = 3, k = 64; in FP64 the values held in
// flight take 104 VGPRs and the readlane form stays faster).
template <typename T, int MODE, int G>
__device__ __forceinline__ void group_rows_lds(const SpmmArgs<T>& a, int32_t row_lane, int64_t start_lane,
                                           int lane, int64_t col, int64_t lc, T* wv) {
    constexpr int U = G >= 4 ? 4 : 8;   // gathers in flight per wave
    const int64_t k = a.k;
    int64_t r[G], st[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
        r[i] = __builtin_amdgcn_readlane(row_lane, i);
        const int lo = __builtin_amdgcn_readlane((int)start_lane, i);
        const int hi = __builtin_amdgcn_readlane((int)(start_lane >> 32), i);
        st[i] = ((int64_t)hi << 32) | (uint32_t)lo;
    }
    const int64_t m = a.rp[r[0] + 1] - st[0];
    T acc[G];
#pragma unroll
    for (int i = 0; i < G; ++i) acc[i] = 0;
    for (int64_t b = 0; b < m; b += BW) {
        const int mb = (int)min((int64_t)BW, m - b);
        const int li = lane < mb ? lane : mb - 1;
        const int32_t cw = a.ci[st[0] + b + li];
#pragma unroll
        for (int i = 0; i < G; ++i) wv[i * BW + lane] = a.val[st[i] + b + li];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int t = 0;
        for (; t + U <= mb; t += U) {
            T xs[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t c = __builtin_amdgcn_readlane(cw, t + u);
                xs[u] = a.v[c * k + lc];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int i = 0; i < G; ++i) acc[i] += wv[i * BW + t + u] * xs[u];
        }
        for (; t < mb; ++t) {
            const int64_t c = __builtin_amdgcn_readlane(cw, t);
            const T x = a.v[c * k + lc];
#pragma unroll
            for (int i = 0; i < G; ++i) acc[i] += wv[i * BW + t] * x;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (col < k) {
#pragma unroll
        for (int i = 0; i < G; ++i) spmm_epilogue<T, MODE>(a, r[i], col, acc[i]);
    }
}

// One wavefront per group of rows with identical column lists (at most
// GROUP_MAX rows; a.gptr / a.grows list them), 64 columns per wave.
template <typename T, int MODE, int WPB>
__global__ void __launch_bounds__(WPB* BW) spmm_group_kernel(SpmmArgs<T> a) {
    if (a.run && *a.run == 0) return;
    const int lane = threadIdx.x % BW;
    const int64_t w = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(threadIdx.x / BW);
    if (w >= a.ngroups) return;
    const int32_t g0 = __builtin_amdgcn_readfirstlane(a.gptr[w]);
    const int g = __builtin_amdgcn_readfirstlane(a.gptr[w + 1]) - g0;
    const int32_t row_lane = a.grows[g0 + (lane < g ? lane : g - 1)];
    const int64_t start_lane = a.rp[row_lane];
    const int64_t col = (int64_t)blockIdx.y * BW + lane;
    const int64_t lc = col < a.k ? col : a.k - 1;
    if constexpr (sizeof(T) == 4) {
        __shared__ T wvals[WPB][GROUP_MAX * BW];
        T* wv = wvals[threadIdx.x / BW];
        switch (g) {
            case 1: group_rows_lds<T, MODE, 1>(a, row_lane, start_lane, lane, col, lc, wv); break;
            case 2: group_rows_lds<T, MODE, 2>(a, row_lane, start_lane, lane, col, lc, wv); break;
            case 3: group_rows_lds<T, MODE, 3>(a, row_lane, start_lane, lane, col, lc, wv); break;
            case 4: group_rows_lds<T, MODE, 4>(a, row_lane, start_lane, lane, col, lc, wv); break;
            case 5: group_rows_lds<T, MODE, 5>(a, row_lane, start_lane, lane, col, lc, wv); break;
            case 6: group_rows_lds<T, MODE, 6>(a, row_lane, start_lane, lane, col, lc, wv); break;
            case 7: group_rows_lds<T, MODE, 7>(a, row_lane, start_lane, lane, col, lc, wv); break;
            default: group_rows_lds<T, MODE, 8>(a, row_lane, start_lane, lane, col, lc, wv); break;
        }
    } else {
        switch (g) {
            case 1: group_rows_readlane<T, MODE, 1>(a, row_lane, start_lane, lane, col, lc); break;
            case 2: group_rows_readlane<T, MODE, 2>(a, row_lane, start_lane, lane, col, lc); break;
            case 3: group_rows_readlane<T, MODE, 3>(a, row_lane, start_lane, lane, col, lc); break;
            case 4: group_rows_readlane<T, MODE, 4>(a, row_lane, start_lane, lane, col, lc); break;
            case 5: group_rows_readlane<T, MODE, 5>(a, row_lane, start_lane, lane, col, lc); break;
            case 6: group_rows_readlane<T, MODE, 6>(a, row_lane, start_lane, lane, col, lc); break;
            case 7: group_rows_readlane<T, MODE, 7>(a, row_lane, start_lane, lane, col, lc); break;
            default: group_rows_readlane<T, MODE, 8>(a, row_lane, start_lane, lane, col, lc); break;
        }
    }
}

// Tile shapes the tuner chooses from.
// kind: 0 spmm_kernel (kt lanes per row), 1 spmm_wave_kernel (one row per
// wavefront), 2 spmm_group_kernel (one row group per wavefront); kinds 1 and
// 2 take 64 columns per wave.
enum TileKind { TILE_LANES = 0, TILE_WAVE = 1, TILE_GROUP = 2 };
struct Tile { int kt, wpb, kind; };
const Tile kTiles[] = {{64, 8, TILE_GROUP}, {64, 4, TILE_GROUP}, {64, 8, TILE_WAVE}, {64, 4, TILE_WAVE},
                       {64, 4, TILE_LANES}, {64, 8, TILE_LANES}, {64, 2, TILE_LANES}, {32, 4, TILE_LANES},
                       {32, 8, TILE_LANES}, {16, 4, TILE_LANES}, {16, 8, TILE_LANES}, {8, 8, TILE_LANES}};

template <typename T, int MODE>
void launch_spmm_tile(const SpmmArgs<T>& a, Tile t, hipStream_t s) {
    if (t.kind == TILE_WAVE || t.kind == TILE_GROUP) {
        const int64_t units = t.kind == TILE_WAVE ? a.n : a.ngroups;
        if (t.kind == TILE_GROUP && (a.gptr == nullptr || a.grows == nullptr))
            throw Error(GIAMG_EINVAL, "row groups missing");
        if (units <= 0) return;
        const dim3 grid((unsigned)((units + t.wpb - 1) / t.wpb), (unsigned)((a.k + BW - 1) / BW));
#define GIAMG_WTILE(KIND, WPB, KERNEL)                                              \
        if (t.kind == KIND && t.wpb == WPB) {                                       \
            KERNEL<T, MODE, WPB><<<grid, dim3(WPB * BW), 0, s>>>(a);                \
            return;                                                                 \
        }
        GIAMG_WTILE(TILE_WAVE, 8, spmm_wave_kernel) GIAMG_WTILE(TILE_WAVE, 4, spmm_wave_kernel)
        GIAMG_WTILE(TILE_GROUP, 8, spmm_group_kernel) GIAMG_WTILE(TILE_GROUP, 4, spmm_group_kernel)
#undef GIAMG_WTILE
        throw Error(GIAMG_EINVAL, "unknown tile");
    }
    const int rpw = BW / t.kt;
    const int64_t rows_per_block = (int64_t)rpw * t.wpb;
    const dim3 grid((unsigned)((a.n + rows_per_block - 1) / rows_per_block),
                    (unsigned)((a.k + t.kt - 1) / t.kt));
    const dim3 block(t.wpb * BW);
#define GIAMG_TILE(KT, WPB)                                                         \
    if (t.kt == KT && t.wpb == WPB) {                                               \
        spmm_kernel<T, MODE, KT, WPB><<<grid, block, 0, s>>>(a);                    \
        return;                                                                     \
    }
    GIAMG_TILE(64, 4) GIAMG_TILE(64, 8) GIAMG_TILE(64, 2) GIAMG_TILE(32, 4)
    GIAMG_TILE(32, 8) GIAMG_TILE(16, 4) GIAMG_TILE(16, 8) GIAMG_TILE(8, 8)
#undef GIAMG_TILE
    throw Error(GIAMG_EINVAL, "unknown tile");
}

template <typename T>
void launch_spmm_any(int mode, const SpmmArgs<T>& a, Tile t, hipStream_t s) {
    if (a.n <= 0) return;
    switch (mode) {
        case SPMV_PLAIN: launch_spmm_tile<T, SPMV_PLAIN>(a, t, s); break;
        case SPMV_RESID: launch_spmm_tile<T, SPMV_RESID>(a, t, s); break;
        case SPMV_ADD: launch_spmm_tile<T, SPMV_ADD>(a, t, s); break;
        case SPMV_CHEB_INIT: launch_spmm_tile<T, SPMV_CHEB_INIT>(a, t, s); break;
        case SPMV_CHEB_STEP: launch_spmm_tile<T, SPMV_CHEB_STEP>(a, t, s); break;
        case SPMV_JACOBI: launch_spmm_tile<T, SPMV_JACOBI>(a, t, s); break;
        default: throw Error(GIAMG_EINVAL, "unknown block product mode");
    }
    GIAMG_HIP(hipGetLastError());
}

// ---- row-local block kernels ------------------------------------------------
template <typename T>
__global__ void bcheb_init0_kernel(int64_t n, int k, const T* __restrict__ f, const T* __restrict__ dinv,
                                   T* __restrict__ r, T* __restrict__ d, T* __restrict__ x, T inv_theta,
                                   int write_x, const int* run) {
    if (run && *run == 0) return;
    const int64_t total = n * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T res = dinv[i / k] * f[i];
        const T dd = res * inv_theta;
        r[i] = res;
        d[i] = dd;
        if (write_x) x[i] = dd;
    }
}

template <typename T>
__global__ void bjacobi0_kernel(int64_t n, int k, const T* __restrict__ f, const T* __restrict__ dinv,
                                T* __restrict__ x, T omega, const int* run) {
    if (run && *run == 0) return;
    const int64_t total = n * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = omega * dinv[i / k] * f[i];
}

template <typename Tin, typename Tout>
__global__ void bconvert_kernel(int64_t total, const Tin* __restrict__ a, Tout* __restrict__ b,
                                int accumulate, const int* run) {
    if (run && *run == 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = accumulate ? (Tout)(b[i] + (Tout)a[i]) : (Tout)a[i];
}

// Y = inv F for the dense coarsest inverse, FP64 accumulation, one row per
// wave.  Each row sums over j in ascending order; the loads of COARSE_U
// consecutive terms are issued before their multiply-adds, so the loop is
// not one L2 round trip per term.
constexpr int COARSE_U = 8;
template <typename T>
__global__ void __launch_bounds__(BW) bcoarse_kernel(int64_t n, int k, const double* __restrict__ inv,
                                                     const T* __restrict__ f, T* __restrict__ y,
                                                     const int* run) {
    if (run && *run == 0) return;
    const int64_t row = blockIdx.x;
    const double* __restrict__ ir = inv + row * n;
    for (int64_t col = threadIdx.x; col < k; col += blockDim.x) {
        double acc = 0.0;
        int64_t j = 0;
        for (; j + COARSE_U <= n; j += COARSE_U) {
            double fv[COARSE_U], iv[COARSE_U];
#pragma unroll
            for (int u = 0; u < COARSE_U; ++u) {
                fv[u] = (double)f[(j + u) * k + col];
                iv[u] = ir[j + u];
            }
#pragma unroll
            for (int u = 0; u < COARSE_U; ++u) acc += iv[u] * fv[u];
        }
        for (; j < n; ++j) acc += ir[j] * (double)f[j * k + col];
        y[row * k + col] = (T)acc;
    }
}

static unsigned bgrid(int64_t total) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

// ---- per-column CG state ------------------------------------------------------
struct ColState {
    double bb, rr, rz, pq, alpha, beta, rznew, zrold;
    int active, iters, status, init;   // init: column being (re)started
};

// ---- column dot products with a fixed row partition ---------------------------
// partial[(c*nb + b)] = sum over rows of block b (in order) of a[i][c] * b[i][c]
// (b FP64, or FP32 widened exactly)
template <typename TB>
__global__ void __launch_bounds__(256) bdot_partial_kernel(int64_t n, int k, const double* __restrict__ a,
                                                           const TB* __restrict__ b,
                                                           double* __restrict__ partial, int64_t nb,
                                                           const int* run) {
    if (run && *run == 0) return;
    __shared__ double sh[4][BW];
    const int lane = threadIdx.x % BW, wave = threadIdx.x / BW;
    const int64_t col = (int64_t)blockIdx.y * BW + lane;
    const int64_t r0 = (int64_t)blockIdx.x * DOT_ROWS + wave * (DOT_ROWS / 4);
    double s = 0.0;
    if (col < k) {
        const int64_t r1 = (r0 + DOT_ROWS / 4 < n) ? r0 + DOT_ROWS / 4 : n;
        for (int64_t i = r0; i < r1; ++i) s += a[i * k + col] * (double)b[i * k + col];
    }
    sh[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && col < k)
        partial[col * nb + blockIdx.x] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

// The same partials for two dots that share b: a.b into partial, a2.b into
// partial2 (each sum in the order of bdot_partial_kernel, so the same bits).
template <typename TB>
__global__ void __launch_bounds__(256) bdot2_partial_kernel(int64_t n, int k, const double* __restrict__ a,
                                                            const double* __restrict__ a2,
                                                            const TB* __restrict__ b,
                                                            double* __restrict__ partial,
                                                            double* __restrict__ partial2, int64_t nb,
                                                            const int* run) {
    if (run && *run == 0) return;
    __shared__ double sh[2][4][BW];
    const int lane = threadIdx.x % BW, wave = threadIdx.x / BW;
    const int64_t col = (int64_t)blockIdx.y * BW + lane;
    const int64_t r0 = (int64_t)blockIdx.x * DOT_ROWS + wave * (DOT_ROWS / 4);
    double s = 0.0, s2 = 0.0;
    if (col < k) {
        const int64_t r1 = (r0 + DOT_ROWS / 4 < n) ? r0 + DOT_ROWS / 4 : n;
        for (int64_t i = r0; i < r1; ++i) {
            const double bi = (double)b[i * k + col];
            s += a[i * k + col] * bi;
            s2 += a2[i * k + col] * bi;
        }
    }
    sh[0][wave][lane] = s;
    sh[1][wave][lane] = s2;
    __syncthreads();
    if (wave == 0 && col < k) {
        partial[col * nb + blockIdx.x] = ((sh[0][0][lane] + sh[0][1][lane]) + sh[0][2][lane]) + sh[0][3][lane];
        partial2[col * nb + blockIdx.x] = ((sh[1][0][lane] + sh[1][1][lane]) + sh[1][2][lane]) + sh[1][3][lane];
    }
}

// field `which` of ColState (0 bb, 1 rr, 2 rznew, 3 zrold, 4 pq)
__device__ __forceinline__ double* state_field(ColState& s, int which) {
    return which == 0 ? &s.bb : which == 1 ? &s.rr : which == 2 ? &s.rznew : which == 3 ? &s.zrold : &s.pq;
}

// Column c's dot = fixed-order sum of partial[set][c*nb + 0..nb), stored into
// field which[set] of its state (only starting columns if only_init); set =
// blockIdx.y, partial sets nb*k apart.  Each column is summed on its own, so
// a column's bits do not depend on k.
__global__ void __launch_bounds__(256) bdot_reduce_kernel(int64_t nb, int k, const double* __restrict__ partial,
                                                          ColState* st, int which0, int which1, int only_init,
                                                          const int* run) {
    if (run && *run == 0) return;
    __shared__ double sh[256 / BW];
    const int64_t c = blockIdx.x;
    const double* __restrict__ p = partial + (int64_t)blockIdx.y * nb * k + c * nb;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += 256) s += p[i];
#pragma unroll
    for (int o = BW / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, BW);
    if (threadIdx.x % BW == 0) sh[threadIdx.x / BW] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
#pragma unroll
        for (int w = 1; w < 256 / BW; ++w) t += sh[w];
        if (!(only_init && !st[c].init)) *state_field(st[c], blockIdx.y == 0 ? which0 : which1) = t;
    }
}


// Starting columns: decide activity from ||b|| and ||r0||; run = any active.
__global__ void bcg_start_kernel(int k, ColState* st, double tol, int* run) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        ColState& s = st[c];
        if (s.init) {
            s.iters = 0;
            s.status = GIAMG_OK;
            s.active = 0;
            if (s.bb > 0.0 && !(sqrt(s.rr) / sqrt(s.bb) < tol)) {
                s.active = 1;
                if (!isfinite(s.rr)) { s.active = 0; s.status = GIAMG_EBREAKDOWN; }
            }
        }
        if (s.active) atomicOr(&any, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *run = any;
}

// Finish starting columns: rz = (r, z), clear the flag.
__global__ void bcg_start_finish_kernel(int k, ColState* st) {
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        ColState& s = st[c];
        if (!s.init) continue;
        if (s.active) {
            s.rz = s.rznew;
            if (!isfinite(s.rz)) { s.active = 0; s.status = GIAMG_EBREAKDOWN; }
        }
        s.init = 0;
    }
}

// dst = src on starting columns
__global__ void bcopy_init_kernel(int64_t n, int k, const double* __restrict__ src, double* __restrict__ dst,
                                  const ColState* __restrict__ st) {
    const int64_t total = n * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        if (st[i % k].init) dst[i] = src[i];
}

__global__ void bcg_alpha_kernel(int k, ColState* st, const int* run) {
    if (*run == 0) return;
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        ColState& s = st[c];
        if (!s.active) { s.alpha = 0.0; continue; }
        if (!(s.pq > 0.0) || !isfinite(s.pq) || !isfinite(s.rz)) {
            s.active = 0;
            s.status = GIAMG_EBREAKDOWN;
            s.alpha = 0.0;
        } else {
            s.alpha = s.rz / s.pq;
        }
    }
}

// x += alpha p; r_old = r; r -= alpha q   (active columns only)
// x += alpha p, r_old = r, r -= alpha q for the active columns, and the
// partials of r.r of every column on the row partition and in the order of
// bdot_partial_kernel (so the same bits as that kernel run after this one).
// r32 (mixed precision): every column's r rounded to FP32, the V-cycle input.
// dinvc set: also level 0's zero-start Chebyshev init of the next V-cycle
// (cr = dinvc f, cd = cr inv_theta with f the V-cycle input in TC: the
// operations of bcheb_init0_kernel<TC>, so the same bits).
template <typename TC>
__global__ void __launch_bounds__(256) bcg_update_kernel(int64_t n, int k, double* __restrict__ x,
                                                         double* __restrict__ r, double* __restrict__ rold,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ q,
                                                         const ColState* __restrict__ st,
                                                         float* __restrict__ r32,
                                                         const TC* __restrict__ dinvc, TC* __restrict__ cr,
                                                         TC* __restrict__ cd, TC inv_theta,
                                                         double* __restrict__ partial, int64_t nb,
                                                         const int* run) {
    if (*run == 0) return;
    __shared__ double sh[4][BW];
    const int lane = threadIdx.x % BW, wave = threadIdx.x / BW;
    const int64_t col = (int64_t)blockIdx.y * BW + lane;
    const int64_t r0 = (int64_t)blockIdx.x * DOT_ROWS + wave * (DOT_ROWS / 4);
    double s = 0.0;
    if (col < k) {
        const bool active = st[col].active != 0;
        const double alpha = st[col].alpha;
        const int64_t r1 = (r0 + DOT_ROWS / 4 < n) ? r0 + DOT_ROWS / 4 : n;
        for (int64_t i = r0; i < r1; ++i) {
            const int64_t idx = i * k + col;
            double rn = r[idx];
            if (active) {
                x[idx] += alpha * p[idx];
                if (rold) rold[idx] = rn;
                rn = rn - alpha * q[idx];
                r[idx] = rn;
            }
            if (r32) r32[idx] = (float)rn;
            if (dinvc) {
                const TC res = dinvc[i] * (TC)rn;
                cr[idx] = res;
                cd[idx] = res * inv_theta;
            }
            s += rn * rn;
        }
    }
    sh[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && col < k)
        partial[col * nb + blockIdx.x] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

__global__ void bcg_check_kernel(int k, ColState* st, double tol, int maxit, int* run) {
    __shared__ int any;
    if (*run == 0) return;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        ColState& s = st[c];
        if (s.active) {
            s.iters += 1;
            const double rel = sqrt(s.rr) / sqrt(s.bb);
            if (!isfinite(rel)) {
                s.active = 0;
                s.status = GIAMG_EBREAKDOWN;
            } else if (rel < tol) {
                s.active = 0;
                s.status = GIAMG_OK;
            } else if (s.iters >= maxit) {
                s.active = 0;
                s.status = GIAMG_ENOTCONV;
            }
        }
        if (s.active) atomicOr(&any, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *run = any;
}

__global__ void bcg_beta_kernel(int k, ColState* st, int flexible, const int* run) {
    if (*run == 0) return;
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        ColState& s = st[c];
        if (!s.active) continue;
        const double rzn = s.rznew;
        s.beta = flexible ? (rzn - s.zrold) / s.rz : rzn / s.rz;
        if (!isfinite(rzn)) {
            s.active = 0;
            s.status = GIAMG_EBREAKDOWN;
        }
        s.rz = rzn;
    }
}

// p = z + beta p (first: p = z), active columns only; z FP64, or the FP32
// V-cycle output widened exactly
template <typename TZ>
__global__ void bcg_direction_kernel(int64_t n, int k, const TZ* __restrict__ z, double* __restrict__ p,
                                     const ColState* __restrict__ st, int first, const int* run) {
    if (*run == 0) return;
    const int64_t total = n * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const ColState& s = st[i % k];
        if (!s.active || (first && !s.init)) continue;
        const double zi = (double)z[i];
        p[i] = first ? zi : zi + s.beta * p[i];
    }
}

// x = 0 for right-hand sides that are identically zero
__global__ void bzero_cols_kernel(int64_t n, int k, double* __restrict__ x, const ColState* __restrict__ st) {
    const int64_t total = n * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        if (st[i % k].init && st[i % k].bb == 0.0) x[i] = 0.0;
}

__global__ void bfill_state_kernel(int k, ColState* st) {
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        ColState z{};
        z.init = 1;
        st[c] = z;
    }
}

// (re)start the listed slots: zero their state, mark them starting
__global__ void bmark_init_kernel(int k, ColState* st, const int* slots, int ns) {
    for (int i = threadIdx.x; i < ns; i += blockDim.x) {
        const int c = slots[i];
        if (c < 0 || c >= k) continue;
        ColState z{};
        z.init = 1;
        st[c] = z;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// per-handle batch workspace
// ---------------------------------------------------------------------------
struct BatchLevel {
    DevBuf<double> f, x, r, d0, d1, t;
    DevBuf<float> f32, x32, r32, d032, d132, t32;
};

// Rows of one operator with identical column lists, split into groups of at
// most GROUP_MAX rows (near-equal sizes): rows[ptr[g] .. ptr[g+1]) are group
// g, groups in order of their first row.
struct RowGroups {
    DevBuf<int32_t> ptr, rows;
    int64_t count = 0;
};

struct BatchState {
    int k = 0;
    bool mixed = false;
    std::vector<BatchLevel> lv;
    DevBuf<double> R, Z, P, Q, Rold;
    DevBuf<double> partial;   // [2][k][dot blocks] column-dot partials
    DevBuf<ColState> st;
    DevBuf<int> run;
    std::map<std::string, Tile> tiles;   // tuned tile per operator and precision
    std::map<std::string, RowGroups> groups;   // per operator (pattern only)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const double* graph_b = nullptr;
    double* graph_x = nullptr;
    double graph_tol = -1.0;
    double bytes_iter = 0.0;
    hipStream_t stream = nullptr;     // capturable stream ordered after the caller's
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    ~BatchState() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (stream) (void)hipStreamDestroy(stream);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
    }
};

void BatchDeleter::operator()(BatchState* b) const { delete b; }

std::mutex& capture_mutex() {
    static std::mutex m;
    return m;
}

namespace {

template <typename T> struct BL;
template <> struct BL<double> {
    static double* f(BatchLevel& b) { return b.f.get(); }
    static double* x(BatchLevel& b) { return b.x.get(); }
    static double* r(BatchLevel& b) { return b.r.get(); }
    static double* d0(BatchLevel& b) { return b.d0.get(); }
    static double* d1(BatchLevel& b) { return b.d1.get(); }
    static double* t(BatchLevel& b) { return b.t.get(); }
    static const double* A(const Level& L) { return L.A.val.get(); }
    static const double* P(const Level& L) { return L.P.val.get(); }
    static const double* R(const Level& L) { return L.R.val.get(); }
    static const double* AP(const Level& L) { return L.AP.val.get(); }
    static const double* dinv(const Level& L) { return L.dinv.get(); }
};
template <> struct BL<float> {
    static float* f(BatchLevel& b) { return b.f32.get(); }
    static float* x(BatchLevel& b) { return b.x32.get(); }
    static float* r(BatchLevel& b) { return b.r32.get(); }
    static float* d0(BatchLevel& b) { return b.d032.get(); }
    static float* d1(BatchLevel& b) { return b.d132.get(); }
    static float* t(BatchLevel& b) { return b.t32.get(); }
    static const float* A(const Level& L) { return L.A.val32.get(); }
    static const float* P(const Level& L) { return L.P.val32.get(); }
    static const float* R(const Level& L) { return L.R.val32.get(); }
    static const float* AP(const Level& L) { return L.AP.val32.get(); }
    static const float* dinv(const Level& L) { return L.dinv32.get(); }
};

template <typename T>
SpmmArgs<T> bargs(const DevCSR& M, const T* val, int k, const int* run) {
    SpmmArgs<T> a;
    a.rp = M.rp.get(); a.ci = M.ci.get(); a.val = val; a.n = M.nrows; a.k = k; a.run = run;
    return a;
}

struct BatchCtx {
    Handle& H;
    BatchState& B;
    int k;
    const int* run;
    bool count_bytes;
    hipStream_t s() const { return B.stream; }
};

double spmm_bytes(const DevCSR& M, int k, double vb, double rowvecs) {
    return (vb + 4.0) * M.nnz + 8.0 * (M.nrows + 1) + vb * (double)M.ncols * k +
           rowvecs * vb * (double)M.nrows * k;
}

// Group the rows of M by identical column lists (host pass over the
// pattern), groups in the order of their first rows.  (Groups in Z-order of
// their elements, with each XCD taking a contiguous range of them, raised
// the L2 hit rate of the block products from 0.55 to 0.88 and cut their L2
// misses fourfold, but measured 2-3 % slower: the products are not bound by
// the misses.)
RowGroups build_row_groups(const DevCSR& M, hipStream_t s) {
    RowGroups G;
    const int64_t n = M.nrows;
    if (n <= 0) return G;
    std::vector<int64_t> rp((size_t)n + 1);
    std::vector<int32_t> ci((size_t)M.nnz);
    GIAMG_HIP(hipMemcpyAsync(rp.data(), M.rp.get(), rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (M.nnz > 0)
        GIAMG_HIP(hipMemcpyAsync(ci.data(), M.ci.get(), ci.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    std::vector<std::vector<int32_t>> groups;
    for (const auto& c : identical_row_classes(rp, ci, n)) {   // ceil(size / GROUP_MAX) near-equal groups
        const size_t parts = (c.size() + GROUP_MAX - 1) / GROUP_MAX;
        for (size_t q = 0; q < parts; ++q)
            groups.emplace_back(c.begin() + c.size() * q / parts, c.begin() + c.size() * (q + 1) / parts);
    }
    std::sort(groups.begin(), groups.end(),
              [](const std::vector<int32_t>& a, const std::vector<int32_t>& b) { return a.front() < b.front(); });
    std::vector<int32_t> ptr{0}, rows;
    rows.reserve((size_t)n);
    for (auto& g : groups) {
        rows.insert(rows.end(), g.begin(), g.end());
        ptr.push_back((int32_t)rows.size());
    }
    G.count = (int64_t)groups.size();
    G.ptr = DevBuf<int32_t>(ptr.size());
    G.rows = DevBuf<int32_t>(rows.size());
    GIAMG_HIP(hipMemcpyAsync(G.ptr.get(), ptr.data(), ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(G.rows.get(), rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    return G;
}

const RowGroups& row_groups(BatchCtx& c, const DevCSR& M, const std::string& key) {
    auto it = c.B.groups.find(key);
    if (it == c.B.groups.end()) it = c.B.groups.emplace(key, build_row_groups(M, c.s())).first;
    return it->second;
}

template <typename T>
void with_groups(BatchCtx& c, const DevCSR& M, const std::string& key, Tile t, SpmmArgs<T>& a) {
    if (t.kind != TILE_GROUP) return;
    const RowGroups& G = row_groups(c, M, key);
    a.gptr = G.ptr.get();
    a.grows = G.rows.get();
    a.ngroups = G.count;
}

// tile lookup (tuned on first use, outside any capture)
template <typename T>
Tile tile_for(BatchCtx& c, const DevCSR& M, const std::string& key);

template <typename T>
void spmm(BatchCtx& c, int mode, const DevCSR& M, SpmmArgs<T> a, const std::string& key,
          double rowvecs) {
    const Tile t = tile_for<T>(c, M, key);
    if (c.count_bytes) c.H.bytes += spmm_bytes(M, c.k, sizeof(T), rowvecs);
    with_groups<T>(c, M, key, t, a);
    launch_spmm_any<T>(mode, a, t, c.s());
}

template <typename T>
Tile tile_for(BatchCtx& c, const DevCSR& M, const std::string& key) {
    const std::string full = key + (sizeof(T) == 4 ? "/f32" : "/f64");
    auto it = c.B.tiles.find(full);
    if (it != c.B.tiles.end()) return it->second;
    // tune: time a plain product of this operator for every tile shape
    DevBuf<T> xin((size_t)std::max<int64_t>(M.ncols, 1) * c.k), yout((size_t)std::max<int64_t>(M.nrows, 1) * c.k);
    GIAMG_HIP(hipMemsetAsync(xin.get(), 0, xin.n * sizeof(T), c.s()));
    const T* val = nullptr;
    if constexpr (sizeof(T) == 4) val = M.val32.get(); else val = M.val.get();
    SpmmArgs<T> a;
    a.rp = M.rp.get(); a.ci = M.ci.get(); a.val = val; a.n = M.nrows; a.k = c.k;
    a.v = xin.get(); a.y = yout.get();
    Tile best = kTiles[0];
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    GIAMG_HIP(hipEventCreate(&e0));
    GIAMG_HIP(hipEventCreate(&e1));
    // GIAMG_BATCH_LANES / WAVE / GROUP force TILE_LANES / WAVE / GROUP
    const int want = c.H.opts.batch_kernel - GIAMG_BATCH_LANES;
    for (const Tile& t : kTiles) {
        if (want >= 0 ? t.kind != want : (t.kt > 2 * c.k && t.kt > 8)) continue;   // forced / idle lanes
        with_groups<T>(c, M, key, t, a);
        launch_spmm_any<T>(SPMV_PLAIN, a, t, c.s());
        GIAMG_HIP(hipEventRecord(e0, c.s()));
        for (int i = 0; i < 3; ++i) launch_spmm_any<T>(SPMV_PLAIN, a, t, c.s());
        GIAMG_HIP(hipEventRecord(e1, c.s()));
        GIAMG_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        GIAMG_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c.B.tiles[full] = best;
    return best;
}

// Post-smoothing after the coarse correction x = x' + P e takes the residual
// t = f - A x' and e: its first product is t - (A P) e.
template <typename T>
void bsmooth(BatchCtx& c, size_t l, const T* f, T* x, bool zero_start, const T* t = nullptr,
             const T* e = nullptr, bool init_done = false) {
    Handle& H = c.H;
    Level& L = H.levels[l];
    BatchLevel& W = c.B.lv[l];
    const int k = c.k;
    const int deg = H.opts.degree;
    const std::string key = "A" + std::to_string(l);
    const int64_t total = L.n * (int64_t)k;
    if (H.opts.smoother == GIAMG_SMOOTHER_JACOBI) {
        const T w = (T)H.opts.omega;
        T* buf[2] = {x, BL<T>::d0(W)};
        int cur = 0, start = 0;
        if (zero_start) {
            if (c.count_bytes) H.bytes += 3.0 * sizeof(T) * total;
            bjacobi0_kernel<T><<<bgrid(total), 256, 0, c.s()>>>(L.n, k, f, BL<T>::dinv(L), x, w, c.run);
            start = 1;
        }
        for (int s = start; s < deg; ++s) {
            SpmmArgs<T> a = bargs<T>(L.A, BL<T>::A(L), k, c.run);
            a.v = buf[cur]; a.y = buf[1 - cur]; a.f = f; a.dinv = BL<T>::dinv(L); a.omega = w;
            spmm<T>(c, SPMV_JACOBI, L.A, a, key, 3);
            cur = 1 - cur;
        }
        if (cur == 1) {
            if (c.count_bytes) H.bytes += 2.0 * sizeof(T) * total;
            bconvert_kernel<T, T><<<bgrid(total), 256, 0, c.s()>>>(total, buf[1], x, 0, c.run);
        }
        return;
    }
    const double lo = H.opts.cheb_lo * L.lam_hat, hi = H.opts.cheb_hi * L.lam_hat;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    T* r = BL<T>::r(W);
    T* d[2] = {BL<T>::d0(W), BL<T>::d1(W)};
    if (zero_start) {
        if (!init_done) {
            if (c.count_bytes) H.bytes += (deg == 1 ? 5.0 : 4.0) * sizeof(T) * total;
            bcheb_init0_kernel<T><<<bgrid(total), 256, 0, c.s()>>>(L.n, k, f, BL<T>::dinv(L), r, d[0], x,
                                                                    (T)(1.0 / theta), deg == 1, c.run);
        }
    } else {
        const bool ap = e != nullptr;
        const DevCSR& M = ap ? L.AP : L.A;
        SpmmArgs<T> a = bargs<T>(M, ap ? BL<T>::AP(L) : BL<T>::A(L), k, c.run);
        a.v = ap ? e : x; a.f = ap ? t : f; a.r = r; a.y = d[0]; a.dinv = BL<T>::dinv(L);
        a.inv_theta = (T)(1.0 / theta);
        spmm<T>(c, SPMV_CHEB_INIT, M, a, ap ? "AP" + std::to_string(l) : key, 4);
        if (deg == 1) {
            if (c.count_bytes) H.bytes += 3.0 * sizeof(T) * total;
            bconvert_kernel<T, T><<<bgrid(total), 256, 0, c.s()>>>(total, d[0], x, 1, c.run);
        }
    }
    double rho = 1.0 / sigma;
    for (int j = 1; j < deg; ++j) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        SpmmArgs<T> a = bargs<T>(L.A, BL<T>::A(L), k, c.run);
        a.v = d[(j - 1) & 1]; a.y = d[j & 1]; a.r = r; a.x = x; a.dinv = BL<T>::dinv(L);
        a.c1 = (T)(rn * rho); a.c2 = (T)(2.0 * rn / delta);
        a.flags = (j == deg - 1 ? CHEB_LAST : 0) | ((zero_start && j == 1) ? CHEB_ASSIGN : 0);
        spmm<T>(c, SPMV_CHEB_STEP, L.A, a, key, (zero_start && j == 1) ? 5 : 6);
        rho = rn;
    }
}

// init_done: level l's zero-start smoother init was written with f (fused).
template <typename T>
void bvcycle(BatchCtx& c, size_t l, const T* f, T* x, bool init_done = false) {
    Handle& H = c.H;
    Level& L = H.levels[l];
    const int k = c.k;
    if (l + 1 == H.levels.size()) {
        if (c.count_bytes) H.bytes += 8.0 * H.nc * H.nc + 2.0 * sizeof(T) * H.nc * k;
        if (H.nc > 0)
            bcoarse_kernel<T><<<(unsigned)H.nc, BW, 0, c.s()>>>(H.nc, k, H.coarse_inv.get(), f, x, c.run);
        return;
    }
    BatchLevel& W = c.B.lv[l];
    BatchLevel& WC = c.B.lv[l + 1];
    const std::string sl = std::to_string(l);
    bsmooth<T>(c, l, f, x, true, nullptr, nullptr, init_done);
    {
        SpmmArgs<T> a = bargs<T>(L.A, BL<T>::A(L), k, c.run);
        a.v = x; a.f = f; a.y = BL<T>::t(W);
        spmm<T>(c, SPMV_RESID, L.A, a, "A" + sl, 2);
    }
    {
        SpmmArgs<T> a = bargs<T>(L.R, BL<T>::R(L), k, c.run);
        a.v = BL<T>::t(W); a.y = BL<T>::f(WC);
        spmm<T>(c, SPMV_PLAIN, L.R, a, "R" + sl, 1);
    }
    bvcycle<T>(c, l + 1, BL<T>::f(WC), BL<T>::x(WC));
    {
        SpmmArgs<T> a = bargs<T>(L.P, BL<T>::P(L), k, c.run);
        a.v = BL<T>::x(WC); a.y = x;
        spmm<T>(c, SPMV_ADD, L.P, a, "P" + sl, 2);
    }
    bsmooth<T>(c, l, f, x, false, BL<T>::t(W), BL<T>::x(WC));
}

// z = V(r).  Mixed precision: the FP32 V-cycle runs on level 0's f32 block
// (r rounded; r32_ready: the CG update already wrote it) and z stays in FP32
// in level 0's x32 block, which the dots and the direction update read
// (widened exactly, so the same values as an FP64 copy).
// init_done: the CG update also wrote level 0's smoother init.
void bprecondition(BatchCtx& c, const double* r, bool r32_ready, bool init_done) {
    const int64_t total = c.H.n_nodes * (int64_t)c.k;
    if (c.B.mixed) {
        BatchLevel& W = c.B.lv[0];
        if (!r32_ready) {
            if (c.count_bytes) c.H.bytes += 12.0 * total;
            bconvert_kernel<double, float><<<bgrid(total), 256, 0, c.s()>>>(total, r, W.f32.get(), 0, c.run);
        }
        bvcycle<float>(c, 0, W.f32.get(), W.x32.get(), init_done);
    } else {
        bvcycle<double>(c, 0, r, c.B.Z.get(), init_done);
    }
}

// The zero-start Chebyshev init of level 0 can ride on the CG update
// (Chebyshev smoother of degree >= 2, a hierarchy of two levels or more).
bool bfused_init(const Handle& H) {
    return H.opts.smoother == GIAMG_SMOOTHER_CHEBYSHEV && H.opts.degree >= 2 && H.levels.size() > 1;
}

// 1 / theta of a level's Chebyshev interval (as bsmooth computes it)
double binv_theta(const Handle& H, const Level& L) {
    const double lo = H.opts.cheb_lo * L.lam_hat, hi = H.opts.cheb_hi * L.lam_hat;
    return 1.0 / (0.5 * (hi + lo));
}

// f(z) with z of the last preconditioner application: FP64 B.Z, or FP32
// level-0 x32 in mixed precision
template <typename F>
void with_z(BatchCtx& c, F&& f) {
    if (c.B.mixed)
        f(static_cast<const float*>(c.B.lv[0].x32.get()));
    else
        f(static_cast<const double*>(c.B.Z.get()));
}

template <typename TZ>
void bdirection(BatchCtx& c, const TZ* z, int first) {
    const int64_t total = c.H.n_nodes * (int64_t)c.k;
    if (c.count_bytes) c.H.bytes += (16.0 + sizeof(TZ)) * total;
    bcg_direction_kernel<TZ><<<bgrid(total), 256, 0, c.s()>>>(c.H.n_nodes, c.k, z, c.B.P.get(), c.B.st.get(),
                                                              first, c.run);
}

int64_t dot_blocks(int64_t n) { return (n + DOT_ROWS - 1) / DOT_ROWS; }

// reduce `sets` partial sets (from B.partial) into the state fields which0, which1
void breduce(BatchCtx& c, int sets, int which0, int which1, int only_init) {
    const int64_t nb = dot_blocks(c.H.n_nodes);
    bdot_reduce_kernel<<<dim3((unsigned)c.k, (unsigned)sets), 256, 0, c.s()>>>(
        nb, c.k, c.B.partial.get(), c.B.st.get(), which0, which1, only_init, c.run);
}

// column dots a.b into the state field `which` (only starting columns if only_init)
template <typename TB>
void bdots(BatchCtx& c, const double* a, const TB* b, int which, int only_init = 0) {
    const int64_t n = c.H.n_nodes;
    const int64_t nb = dot_blocks(n);
    if (c.count_bytes) c.H.bytes += (8.0 + sizeof(TB)) * n * c.k;
    bdot_partial_kernel<TB><<<dim3((unsigned)nb, (unsigned)((c.k + BW - 1) / BW)), 256, 0, c.s()>>>(
        n, c.k, a, b, c.B.partial.get(), nb, c.run);
    breduce(c, 1, which, which, only_init);
}

// a.b into `which` and a2.b into `which2`, reading b once
template <typename TB>
void bdots2(BatchCtx& c, const double* a, const double* a2, const TB* b, int which, int which2) {
    const int64_t n = c.H.n_nodes;
    const int64_t nb = dot_blocks(n);
    if (c.count_bytes) c.H.bytes += (16.0 + sizeof(TB)) * n * c.k;
    double* part = c.B.partial.get();
    bdot2_partial_kernel<TB><<<dim3((unsigned)nb, (unsigned)((c.k + BW - 1) / BW)), 256, 0, c.s()>>>(
        n, c.k, a, a2, b, part, part + nb * c.k, nb, c.run);
    breduce(c, 2, which, which2, 0);
}

void bproduct_A0(BatchCtx& c, int mode, const double* v, const double* f, double* y, double rowvecs) {
    Level& L0 = c.H.levels[0];
    SpmmArgs<double> a = bargs<double>(L0.A, L0.A.val.get(), c.k, c.run);
    a.v = v; a.f = f; a.y = y;
    spmm<double>(c, mode, L0.A, a, "A0", rowvecs);
}

// one CG iteration on the device (captured into the graph)
void iteration(BatchCtx& c, double* X, double tol) {
    Handle& H = c.H;
    BatchState& B = c.B;
    const int64_t total = H.n_nodes * (int64_t)c.k;
    const int maxit = H.opts.maxit;
    const unsigned cb = (unsigned)std::min(c.k, MAX_K);
    bproduct_A0(c, SPMV_PLAIN, B.P.get(), nullptr, B.Q.get(), 1);
    bdots(c, B.P.get(), B.Q.get(), 4);
    bcg_alpha_kernel<<<1, cb, 0, c.s()>>>(c.k, B.st.get(), c.run);
    if (c.count_bytes) H.bytes += (B.mixed ? 60.0 : 48.0) * total;
    const int64_t nb = dot_blocks(H.n_nodes);
    const bool fuse = bfused_init(H);
    const dim3 ug((unsigned)nb, (unsigned)((c.k + BW - 1) / BW));
    Level& L0 = H.levels[0];
    BatchLevel& W0 = B.lv[0];
    const double it0 = binv_theta(H, L0);
    if (B.mixed) {
        if (c.count_bytes && fuse) H.bytes += 8.0 * total;
        bcg_update_kernel<float><<<ug, 256, 0, c.s()>>>(
            H.n_nodes, c.k, X, B.R.get(), B.Rold.get(), B.P.get(), B.Q.get(), B.st.get(), W0.f32.get(),
            fuse ? L0.dinv32.get() : nullptr, W0.r32.get(), W0.d032.get(), (float)it0, B.partial.get(), nb,
            c.run);
    } else {
        if (c.count_bytes && fuse) H.bytes += 16.0 * total;
        bcg_update_kernel<double><<<ug, 256, 0, c.s()>>>(
            H.n_nodes, c.k, X, B.R.get(), nullptr, B.P.get(), B.Q.get(), B.st.get(), nullptr,
            fuse ? L0.dinv.get() : nullptr, W0.r.get(), W0.d0.get(), it0, B.partial.get(), nb, c.run);
    }
    breduce(c, 1, 1, 1, 0);   // r.r
    bcg_check_kernel<<<1, cb, 0, c.s()>>>(c.k, B.st.get(), tol, maxit, B.run.get());
    bprecondition(c, B.R.get(), true, fuse);
    with_z(c, [&](auto z) {
        if (B.mixed)
            bdots2(c, B.R.get(), B.Rold.get(), z, 2, 3);
        else
            bdots(c, B.R.get(), z, 2);
        bcg_beta_kernel<<<1, cb, 0, c.s()>>>(c.k, B.st.get(), B.mixed ? 1 : 0, c.run);
        bdirection(c, z, 0);
    });
    GIAMG_HIP(hipGetLastError());
}

std::unique_ptr<BatchState> make_state(Handle& H, int k) {
    std::unique_ptr<BatchState> B(new BatchState());
    B->k = k;
    B->mixed = H.opts.precision == GIAMG_PREC_MIXED;
    for (auto& L : H.levels) {
        BatchLevel W;
        const size_t m = (size_t)std::max<int64_t>(L.n, 1) * k;
        if (B->mixed) {
            W.f32.alloc(m); W.x32.alloc(m); W.r32.alloc(m); W.d032.alloc(m); W.d132.alloc(m); W.t32.alloc(m);
        } else {
            W.f.alloc(m); W.x.alloc(m); W.r.alloc(m); W.d0.alloc(m); W.d1.alloc(m); W.t.alloc(m);
        }
        B->lv.push_back(std::move(W));
    }
    const size_t tot = (size_t)H.n_nodes * k;
    B->R.alloc(tot); B->P.alloc(tot); B->Q.alloc(tot);
    if (!B->mixed) B->Z.alloc(tot);   // mixed precision: z stays in level 0's x32
    if (B->mixed) B->Rold.alloc(tot);
    const int64_t nb = (H.n_nodes + DOT_ROWS - 1) / DOT_ROWS;
    B->partial.alloc((size_t)nb * k * 2);
    B->st.alloc(k);
    B->run.alloc(1);
    // the caller's stream may be the legacy default stream, which cannot be
    // captured: batched work runs on a stream of its own, ordered by events
    GIAMG_HIP(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking));
    GIAMG_HIP(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    GIAMG_HIP(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
    return B;
}

void ensure_state(Handle& H, int k) {
    if (H.batch && H.batch->k == k) return;
    H.batch.reset();
    H.batch.reset(make_state(H, k).release());
}

// Start the columns flagged `init` without touching the others (their
// recursive residuals and directions stay as they are).
void start_columns(BatchCtx& c, const double* Bm, double* X, double tol) {
    Handle& H = c.H;
    BatchState& B = c.B;
    hipStream_t s = c.s();
    const int k = c.k;
    const int64_t total = H.n_nodes * (int64_t)k;
    const unsigned cb = (unsigned)std::min(k, MAX_K);
    GIAMG_HIP(hipMemsetAsync(B.run.get(), 0xff, sizeof(int), s));
    bproduct_A0(c, SPMV_RESID, X, Bm, B.Q.get(), 2);
    bcopy_init_kernel<<<bgrid(total), 256, 0, s>>>(H.n_nodes, k, B.Q.get(), B.R.get(), B.st.get());
    bdots(c, Bm, Bm, 0, 1);
    bdots(c, B.R.get(), B.R.get(), 1, 1);
    bcg_start_kernel<<<1, cb, 0, s>>>(k, B.st.get(), tol, B.run.get());
    bzero_cols_kernel<<<bgrid(total), 256, 0, s>>>(H.n_nodes, k, X, B.st.get());
    bprecondition(c, B.R.get(), false, false);
    with_z(c, [&](auto z) {
        bdots(c, B.R.get(), z, 2, 1);
        bdirection(c, z, 1);
    });
    bcg_start_finish_kernel<<<1, cb, 0, s>>>(k, B.st.get());
    GIAMG_HIP(hipGetLastError());
}

void tune_all(Handle& H, BatchState& B, int k) {
    BatchCtx t{H, B, k, nullptr, false};
    for (size_t l = 0; l < H.levels.size(); ++l) {
        Level& L = H.levels[l];
        const std::string sl = std::to_string(l);
        tile_for<double>(t, L.A, "A" + sl);
        if (l + 1 == H.levels.size()) continue;
        const bool ap = H.opts.smoother == GIAMG_SMOOTHER_CHEBYSHEV;
        if (B.mixed) {
            tile_for<float>(t, L.A, "A" + sl);
            tile_for<float>(t, L.R, "R" + sl);
            tile_for<float>(t, L.P, "P" + sl);
            if (ap) tile_for<float>(t, L.AP, "AP" + sl);
        } else {
            tile_for<double>(t, L.R, "R" + sl);
            tile_for<double>(t, L.P, "P" + sl);
            if (ap) tile_for<double>(t, L.AP, "AP" + sl);
        }
    }
}

}  // namespace

int solve_batch(Handle& H, const double* Bm, double* X, int32_t k, double tol, giamg_info* infos) {
    AllocStreamScope alloc_scope(H.stream);
    GIAMG_REQUIRE(k <= MAX_K, "at most 1024 right-hand sides per call");
    ensure_state(H, k);
    BatchState& B = *H.batch;
    hipStream_t s = B.stream;
    GIAMG_HIP(hipEventRecord(B.ev_in, H.stream));
    GIAMG_HIP(hipStreamWaitEvent(s, B.ev_in, 0));
    const unsigned cb = (unsigned)std::min(k, MAX_K);
    BatchCtx c{H, B, k, B.run.get(), true};
    H.bytes = 0.0;
    // tune every operator before anything is captured
    tune_all(H, B, k);
    hipEvent_t t0, t1;
    GIAMG_HIP(hipEventCreate(&t0));
    GIAMG_HIP(hipEventCreate(&t1));
    GIAMG_HIP(hipEventRecord(t0, s));
    // start every column: r = b - A x, norms, activity, z = V(r), rz, p = z
    GIAMG_HIP(hipMemsetAsync(B.run.get(), 0xff, sizeof(int), s));   // run everything
    bfill_state_kernel<<<1, cb, 0, s>>>(k, B.st.get());
    start_columns(c, Bm, X, tol);
    const double bytes_start = H.bytes;
    // capture one iteration (pointers are fixed for this k and these b, x)
    if (!B.exec || B.graph_b != Bm || B.graph_x != X || B.graph_tol != tol) {
        if (B.exec) { (void)hipGraphExecDestroy(B.exec); B.exec = nullptr; }
        if (B.graph) { (void)hipGraphDestroy(B.graph); B.graph = nullptr; }
        std::lock_guard<std::mutex> cap(capture_mutex());
        GIAMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
        try {
            iteration(c, X, tol);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        GIAMG_HIP(hipStreamEndCapture(s, &B.graph));
        GIAMG_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
        B.graph_b = Bm;
        B.graph_x = X;
        B.graph_tol = tol;
        B.bytes_iter = H.bytes - bytes_start;
    }
    const double bytes_iter = B.bytes_iter;
    int host_run = 1;
    int launched = 0;
    while (launched < H.opts.maxit) {
        GIAMG_HIP(hipMemcpyAsync(&host_run, B.run.get(), sizeof(int), hipMemcpyDeviceToHost, s));
        GIAMG_HIP(hipStreamSynchronize(s));
        if (!host_run) break;
        const int n = std::min(CHUNK, H.opts.maxit - launched);
        for (int i = 0; i < n; ++i) GIAMG_HIP(hipGraphLaunch(B.exec, s));
        launched += n;
    }
    GIAMG_HIP(hipEventRecord(t1, s));
    std::vector<ColState> hs(k);
    GIAMG_HIP(hipMemcpyAsync(hs.data(), B.st.get(), k * sizeof(ColState), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    float ms = 0.0f;
    GIAMG_HIP(hipEventElapsedTime(&ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    // true residuals (outside the timed region)
    GIAMG_HIP(hipMemsetAsync(B.run.get(), 0xff, sizeof(int), s));
    BatchCtx nc{H, B, k, nullptr, false};
    bproduct_A0(nc, SPMV_RESID, X, Bm, B.Q.get(), 2);
    bdots(nc, B.Q.get(), B.Q.get(), 1);
    std::vector<ColState> ht(k);
    GIAMG_HIP(hipMemcpyAsync(ht.data(), B.st.get(), k * sizeof(ColState), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipEventRecord(B.ev_out, s));
    GIAMG_HIP(hipStreamWaitEvent(H.stream, B.ev_out, 0));
    GIAMG_HIP(hipStreamSynchronize(s));
    int worst = GIAMG_OK;
    int max_iters = 0;
    for (int j = 0; j < k; ++j) {
        max_iters = std::max(max_iters, hs[j].iters);
        const int st = hs[j].status;
        if (st < 0) worst = std::min(worst, st);
        else if (worst >= 0) worst = std::max(worst, st);
        if (infos) {
            giamg_info& in = infos[j];
            in.iters = hs[j].iters;
            in.status = st;
            in.relres = hs[j].bb > 0 ? std::sqrt(hs[j].rr) / std::sqrt(hs[j].bb) : 0.0;
            in.true_relres = hs[j].bb > 0 ? std::sqrt(ht[j].rr) / std::sqrt(hs[j].bb) : 0.0;
            in.solve_ms = ms;
            in.bytes = 0.0;
        }
    }
    if (infos) {
        // whole-batch bytes: start + the replays that ran with active columns
        const double bytes = bytes_start + bytes_iter * max_iters;
        for (int j = 0; j < k; ++j) infos[j].bytes = bytes;
    }
    (void)launched;
    return worst;
}


// ---------------------------------------------------------------------------
// continuous-batching sessions: slots join and leave between iterations
// ---------------------------------------------------------------------------
namespace {

__global__ void bclear_state_kernel(int k, ColState* st) {
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        ColState z{};
        st[c] = z;
    }
}

// column `slot` of the block X [n][k] <- b [n]; x column <- 0
__global__ void bscatter_kernel(int64_t n, int k, int slot, const double* __restrict__ b,
                                double* __restrict__ Bm, double* __restrict__ X) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        Bm[i * k + slot] = b[i];
        X[i * k + slot] = 0.0;
    }
}

__global__ void bgather_kernel(int64_t n, int k, int slot, const double* __restrict__ X, double* __restrict__ x) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = X[i * k + slot];
}

__global__ void bfree_slot_kernel(int k, ColState* st, int slot) {
    if (threadIdx.x == 0 && slot >= 0 && slot < k) {
        ColState z{};
        st[slot] = z;
    }
}

}  // namespace

struct Session {
    Handle* H = nullptr;
    std::unique_ptr<BatchState> B;
    int k = 0;
    double tol = 0.0;
    DevBuf<double> Bm, X;
    DevBuf<int> slots;
    hipEvent_t done = nullptr;         // after the last enqueued step (and its state copy)
    hipEvent_t slots_copied = nullptr; // after the last copy out of host_slots
    ColState* host_states = nullptr;   // pinned: column states as of the last step
    int* host_slots = nullptr;         // pinned: slot list of the last admission
    ~Session() {
        if (done) (void)hipEventDestroy(done);
        if (slots_copied) (void)hipEventDestroy(slots_copied);
        if (host_states) (void)hipHostFree(host_states);
        if (host_slots) (void)hipHostFree(host_slots);
    }
};

Session* session_create(Handle& H, int k, double tol) {
    AllocStreamScope alloc_scope(H.stream);
    GIAMG_REQUIRE(k >= 1 && k <= MAX_K, "slots must be in [1, 1024]");
    std::unique_ptr<Session> S(new Session());
    S->H = &H;
    S->k = k;
    S->tol = tol;
    S->B = make_state(H, k);
    BatchState& B = *S->B;
    hipStream_t s = B.stream;
    GIAMG_HIP(hipEventRecord(B.ev_in, H.stream));
    GIAMG_HIP(hipStreamWaitEvent(s, B.ev_in, 0));
    const size_t tot = (size_t)H.n_nodes * k;
    S->Bm.alloc(tot);
    S->X.alloc(tot);
    S->slots.alloc(k);
    GIAMG_HIP(hipMemsetAsync(S->Bm.get(), 0, tot * sizeof(double), s));
    GIAMG_HIP(hipMemsetAsync(S->X.get(), 0, tot * sizeof(double), s));
    for (DevBuf<double>* v : {&B.R, &B.Z, &B.P, &B.Q})
        if (v->get()) GIAMG_HIP(hipMemsetAsync(v->get(), 0, tot * sizeof(double), s));
    bclear_state_kernel<<<1, 256, 0, s>>>(k, B.st.get());
    GIAMG_HIP(hipMemsetAsync(B.run.get(), 0, sizeof(int), s));
    tune_all(H, B, k);
    BatchCtx c{H, B, k, B.run.get(), false};
    {
        std::lock_guard<std::mutex> cap(capture_mutex());
        GIAMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
        try {
            iteration(c, S->X.get(), tol);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        GIAMG_HIP(hipStreamEndCapture(s, &B.graph));
    }
    GIAMG_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    GIAMG_HIP(hipEventCreateWithFlags(&S->done, hipEventDisableTiming));
    GIAMG_HIP(hipEventCreateWithFlags(&S->slots_copied, hipEventDisableTiming));
    GIAMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&S->host_states), k * sizeof(ColState)));
    GIAMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&S->host_slots), k * sizeof(int)));
    std::memset(S->host_states, 0, k * sizeof(ColState));
    GIAMG_HIP(hipEventRecord(S->slots_copied, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    return S.release();
}

void session_destroy(Session* S) {
    if (!S) return;
    if (S->B) (void)hipStreamSynchronize(S->B->stream);
    delete S;
}

// Copy each b (device, n entries) into its slot and start those columns.
void session_admit(Session* S, const int* slot, const double* const* b, int count) {
    BatchState& B = *S->B;
    Handle& H = *S->H;
    hipStream_t s = B.stream;
    GIAMG_REQUIRE(count >= 1 && count <= S->k, "bad admission count");
    std::vector<int> sl(slot, slot + count);
    // the right-hand sides were written on the caller's stream
    GIAMG_HIP(hipEventRecord(B.ev_in, H.stream));
    GIAMG_HIP(hipStreamWaitEvent(s, B.ev_in, 0));
    for (int i = 0; i < count; ++i) {
        GIAMG_REQUIRE(sl[i] >= 0 && sl[i] < S->k, "slot out of range");
        bscatter_kernel<<<bgrid(H.n_nodes), 256, 0, s>>>(H.n_nodes, S->k, sl[i], b[i], S->Bm.get(), S->X.get());
    }
    // the slot list goes through pinned memory, so the copy is asynchronous;
    // the previous admission's copy out of it has finished first
    GIAMG_HIP(hipEventSynchronize(S->slots_copied));
    std::memcpy(S->host_slots, sl.data(), count * sizeof(int));
    GIAMG_HIP(hipMemcpyAsync(S->slots.get(), S->host_slots, count * sizeof(int), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipEventRecord(S->slots_copied, s));
    bmark_init_kernel<<<1, 256, 0, s>>>(S->k, B.st.get(), S->slots.get(), count);
    BatchCtx c{H, B, S->k, B.run.get(), false};
    start_columns(c, S->Bm.get(), S->X.get(), S->tol);
    GIAMG_HIP(hipEventRecord(S->done, s));
}

// Enqueue `iters` CG iterations for every running slot, then a copy of the
// column states to pinned host memory (asynchronous; session_ready tells
// when both are done and session_states reads the copy).
void session_step(Session* S, int iters) {
    for (int i = 0; i < iters; ++i) GIAMG_HIP(hipGraphLaunch(S->B->exec, S->B->stream));
    GIAMG_HIP(hipMemcpyAsync(S->host_states, S->B->st.get(), S->k * sizeof(ColState), hipMemcpyDeviceToHost,
                             S->B->stream));
    GIAMG_HIP(hipEventRecord(S->done, S->B->stream));
}

namespace {
void decode_states(const Session* S, const ColState* hs, int* state, giamg_info* infos) {
    for (int j = 0; j < S->k; ++j) {
        const ColState& c = hs[j];
        state[j] = (c.active || c.init) ? 1 : 0;
        if (infos) {
            infos[j].iters = c.iters;
            infos[j].status = c.status;
            infos[j].relres = c.bb > 0 ? std::sqrt(c.rr) / std::sqrt(c.bb) : 0.0;
            infos[j].true_relres = -1.0;
            infos[j].solve_ms = 0.0;
            infos[j].bytes = 0.0;
        }
    }
}
}  // namespace

// Slot states as of the last completed step (no synchronisation; call after
// session_ready returned true).
void session_states(Session* S, int* state, giamg_info* infos) {
    decode_states(S, S->host_states, state, infos);
}

bool session_ready(Session* S) {
    const hipError_t e = hipEventQuery(S->done);
    if (e == hipSuccess) return true;
    if (e == hipErrorNotReady) return false;
    GIAMG_HIP(e);
    return false;
}

// Slot states: 1 running, 0 otherwise (free or finished: the caller tracks
// occupancy); infos describe every slot.
void session_poll(Session* S, int* state, giamg_info* infos) {
    BatchState& B = *S->B;
    std::vector<ColState> hs(S->k);
    GIAMG_HIP(hipMemcpyAsync(hs.data(), B.st.get(), S->k * sizeof(ColState), hipMemcpyDeviceToHost, B.stream));
    GIAMG_HIP(hipStreamSynchronize(B.stream));
    decode_states(S, hs.data(), state, infos);
}

// Copy the slot's solution to x (device, n entries) and free the slot.
// The same without waiting: x is written in order on the session stream.
void session_retire_async(Session* S, int slot, double* x) {
    GIAMG_REQUIRE(slot >= 0 && slot < S->k, "slot out of range");
    BatchState& B = *S->B;
    Handle& H = *S->H;
    // x may still be in use on the caller's stream
    GIAMG_HIP(hipEventRecord(B.ev_in, H.stream));
    GIAMG_HIP(hipStreamWaitEvent(B.stream, B.ev_in, 0));
    bgather_kernel<<<bgrid(H.n_nodes), 256, 0, B.stream>>>(H.n_nodes, S->k, slot, S->X.get(), x);
    bfree_slot_kernel<<<1, 64, 0, B.stream>>>(S->k, B.st.get(), slot);
    GIAMG_HIP(hipGetLastError());
}

void session_retire(Session* S, int slot, double* x) {
    session_retire_async(S, slot, x);
    GIAMG_HIP(hipStreamSynchronize(S->B->stream));
}

hipStream_t session_stream(Session* S) { return S->B->stream; }

int64_t session_device_bytes(const Session* S) {
    const BatchState& B = *S->B;
    int64_t b = 0;
    for (const auto& l : B.lv)
        b += (int64_t)(l.f.n + l.x.n + l.r.n + l.d0.n + l.d1.n + l.t.n) * 8 +
             (int64_t)(l.f32.n + l.x32.n + l.r32.n + l.d032.n + l.d132.n + l.t32.n) * 4;
    b += (int64_t)(B.R.n + B.Z.n + B.P.n + B.Q.n + B.Rold.n + B.partial.n) * 8;
    b += (int64_t)(S->Bm.n + S->X.n) * 8;
    return b;
}

}  // namespace giamg
