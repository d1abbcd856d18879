// Device kernels of the GIAMG solve phase for gfx950 (CDNA4).
//
// The solve is HBM-bound sparse work: CSR products of the level operators
// (Algorithm 1: smoothing, residual, restriction, prolongation), vector
// updates and dot products of CG.  Design:
//  * a block streams a contiguous run of up to 8192 nonzeros (whole rows)
//    with coalesced non-temporal loads, so the cache keeps the gathered
//    vector, stages the products in LDS and reduces each row with a lane
//    group sized to the operator's mean row length;
//  * blocks remapped so each of the eight XCDs works on a contiguous slice
//    of rows (its L2 then holds the slice of the gathered vector);
//  * every smoother/CG vector update fused into the product's row epilogue;
//  * reductions are two-stage and fixed-order (no floating-point atomics), so
//    results are bitwise reproducible run to run.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace giamg {

constexpr int WAVE = 64;
constexpr int VEC_THREADS = 256;
constexpr int64_t VEC_MAX_BLOCKS = 2048;
constexpr int RED_THREADS = 1024;

// Device stop flag handed to every kernel launched by this thread while a
// StopScope is open (null otherwise): a kernel whose flag reads nonzero
// returns at once, so iterations queued past convergence cost one dispatch
// per kernel and change nothing.
thread_local const int* g_stop = nullptr;

StopScope::StopScope(const int* flag) : prev_(g_stop) { g_stop = flag; }
StopScope::~StopScope() { g_stop = prev_; }

__device__ __forceinline__ bool stopped(const int* stop) { return stop != nullptr && *stop != 0; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// sum over aligned groups of L lanes; every lane of the group gets the sum
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Row sums of groups of L lanes (L = 16, 4 or 1, each group inside one
// 16-lane DPP row): the same butterfly as group_sum<L> -- step k adds the
// value of the lane that differs in bit k, own value first -- done with DPP
// row rotations instead of LDS permutes.  After the step for bit 8 (4, 2)
// every value repeats with period 8 (4, 2) inside the group, so rotating by
// 4 (2, 1) reads exactly the xor partner's value: the sums are the
// butterfly's bit for bit.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                 0xF, 0xF, false));
}
template <int L, typename T>
__device__ __forceinline__ T row_group_sum(T v) {
    static_assert(L == 16 || L == 4 || L == 1, "row groups of 16, 4 or 1 lanes");
    if constexpr (L == 16) {
        v += dpp_move<0x128>(v);   // row_ror:8  (xor 8)
        v += dpp_move<0x124>(v);   // row_ror:4  (xor 4 on period-8 values)
        v += dpp_move<0x122>(v);   // row_ror:2
        v += dpp_move<0x121>(v);   // row_ror:1
    } else if constexpr (L == 4) {
        v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]  (xor 2)
        v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]  (xor 1)
    }
    return v;
}

// Lane gl's share of a row held in LDS, prod[s .. e): the entries gl,
// gl + L, ... added in that order into one accumulator, the LDS reads of up
// to eight of them issued before the adds so their latencies overlap (the
// additions and their order are those of the plain loop).
template <int L, typename T>
__device__ __forceinline__ T lane_row_sum(const T* prod, int s, int e, int gl) {
    T acc = 0;
    int j = s + gl;
    for (; j + 7 * L < e; j += 8 * L) {
        T p[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) p[u] = prod[j + u * L];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += p[u];
    }
    if (j + 3 * L < e) {
        T p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] = prod[j + u * L];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += p[u];
        j += 4 * L;
    }
    for (; j < e; j += L) acc += prod[j];
    return acc;
}

template <typename T>
__device__ __forceinline__ T ldnt(const T* p) {
    return __builtin_nontemporal_load(p);
}

// Load of the matrix stream (values, slots, column ids): non-temporal, or
// plain where PLAIN (FP32 products of operators with at least
// FP32_PLAIN_MIN_NNZ nonzeros, see kernels.h).  Results are the same bits
// either way.
template <bool PLAIN, typename U>
__device__ __forceinline__ U ld_matrix(const U* p) {
    if constexpr (PLAIN) return *p;
    else return __builtin_nontemporal_load(p);
}

void make_row_blocks(const int64_t* rp, int64_t n, int64_t cap, int64_t max_rows, std::vector<int64_t>& blocks,
                     int& lanes) {
    blocks.clear();
    blocks.push_back(0);
    int64_t acc = 0, rows = 0;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t len = rp[r + 1] - rp[r];
        if (rows > 0 && (acc + len > cap || rows == max_rows)) {
            blocks.push_back(r);
            acc = 0;
            rows = 0;
        }
        acc += len;
        ++rows;
    }
    if (n > 0) blocks.push_back(n);
    // 16 lanes only for long rows: a block's rows should take few passes of
    // the row sums (an FP64 block of 8192 nonzeros in rows of 34, the fine
    // A P operator at p = 4, needs four passes of 1024 threads with 16 lanes
    // per row and one with 4)
    const double mean = n > 0 ? (double)rp[n] / (double)n : 0.0;
    lanes = mean > 48 ? 16 : mean > 6 ? 4 : 1;
}

// Row-local operands of an epilogue, loaded before the row sum is known.
template <typename T>
struct RowIn {
    T f, dinv, r, x, v, y;
};

template <typename T, int MODE>
__device__ __forceinline__ void epilogue_load(const SpmvArgs<T>& a, int64_t row, RowIn<T>& in) {
    if constexpr (MODE == SPMV_RESID || MODE == SPMV_CHEB_INIT || MODE == SPMV_JACOBI ||
                  MODE == SPMV_RINIT)
        in.f = a.f[row];
    if constexpr (MODE == SPMV_CHEB_INIT || MODE == SPMV_CHEB_STEP || MODE == SPMV_JACOBI ||
                  MODE == SPMV_DINV || MODE == SPMV_RCHEB0)
        in.dinv = a.dinv[row];
    if constexpr (MODE == SPMV_CHEB_STEP) {
        in.r = a.r[row];
        in.x = (a.flags & CHEB_ASSIGN) ? T(0) : a.x[row];
    }
    if constexpr (MODE == SPMV_CHEB_STEP || MODE == SPMV_JACOBI || MODE == SPMV_DOT)
        in.v = a.v[row];
    if constexpr (MODE == SPMV_ADD) in.y = a.y[row];
}

// Row epilogue: y is (A v)_row.  `dot` collects this row's share of a block
// partial (DOT: v.y; RINIT: f.f in dot, y.y in dot2).
template <typename T, int MODE>
__device__ __forceinline__ void epilogue_store(const SpmvArgs<T>& a, int64_t row, T y,
                                               const RowIn<T>& in, double& dot, double& dot2) {
    if constexpr (MODE == SPMV_PLAIN) {
        a.y[row] = y;
    } else if constexpr (MODE == SPMV_RESID) {
        a.y[row] = in.f - y;
    } else if constexpr (MODE == SPMV_ADD) {
        a.y[row] = in.y + y;
    } else if constexpr (MODE == SPMV_CHEB_INIT) {
        const T res = in.dinv * (in.f - y);
        a.r[row] = res;
        a.y[row] = res * a.inv_theta;
    } else if constexpr (MODE == SPMV_CHEB_STEP) {
        const T rr = in.r - in.dinv * y;
        const T dn = a.c1 * in.v + a.c2 * rr;
        a.r[row] = rr;
        a.y[row] = dn;
        const T inc = (a.flags & CHEB_LAST) ? in.v + dn : in.v;
        a.x[row] = in.x + inc;
    } else if constexpr (MODE == SPMV_RCHEB0) {
        a.y[row] = y;
        const T res = in.dinv * y;
        a.r[row] = res;
        a.x[row] = res * a.inv_theta;
    } else if constexpr (MODE == SPMV_JACOBI) {
        a.y[row] = in.v + a.omega * in.dinv * (in.f - y);
    } else if constexpr (MODE == SPMV_DOT) {
        a.y[row] = y;
        dot += (double)in.v * (double)y;
    } else if constexpr (MODE == SPMV_DINV) {
        a.y[row] = in.dinv * y;
    } else if constexpr (MODE == SPMV_RINIT) {
        const T ri = in.f - y;
        a.y[row] = ri;
        dot += (double)in.f * (double)in.f;
        dot2 += (double)ri * (double)ri;
    }
}

template <int MODE>
constexpr bool has_partials() { return MODE == SPMV_DOT || MODE == SPMV_RINIT; }

// Butterfly sum over the lanes of a wave with partners 32, 16, 8, 4, 2, 1 in
// that order (the order of group_sum<WAVE>): the two steps across 16-lane
// rows by LDS permutes, the four inside each row by DPP rotations
// (row_group_sum<16>).  Every lane ends with the same bits as
// group_sum<WAVE> gives.
__device__ __forceinline__ double wave_butterfly(double v) {
    v += __shfl_xor(v, 32, WAVE);
    v += __shfl_xor(v, 16, WAVE);
    return row_group_sum<16>(v);
}

// Fixed-order block sums of NV (1 or 2) values per thread, valid in thread 0
// only: each wave adds its lanes by the butterfly above, then thread 0 adds
// the waves' sums in wave order.  One barrier; red holds 2 * NT / WAVE
// doubles and may be reused after a further barrier.
template <int NT, int NV>
__device__ __forceinline__ void block_sum_to0(double* red, int tid, double& a, double& b) {
    static_assert(NV == 1 || NV == 2, "one or two sums");
    constexpr int NW = NT / WAVE;
    a = wave_butterfly(a);
    if constexpr (NV == 2) b = wave_butterfly(b);
    if (tid % WAVE == 0) {
        red[tid / WAVE] = a;
        if constexpr (NV == 2) red[NW + tid / WAVE] = b;
    }
    __syncthreads();
    if (tid == 0) {
        a = red[0];
        if constexpr (NV == 2) b = red[NW];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            a += red[w];
            if constexpr (NV == 2) b += red[NW + w];
        }
    }
}

template <int MODE>
constexpr int n_partials() { return MODE == SPMV_RINIT ? 2 : 1; }

// Forms of step 1 of the streaming product (below).  Loads that depend on
// earlier loads are unconditional, from clamped (always valid) indices, and
// only their stores are guarded: guards there split the code into blocks
// that the compiler separates with waits for every load in flight.

// Copy the runs of the gathered vector v that this wave owns (mine of them,
// descriptors in dsc: lane i holds the wave's run i) into LDS, one run (at
// most 64 entries) per load.  One batch copies SB runs: SB loads in flight,
// then the LDS stores.  The first batch is straight-line code that runs even
// in a wave without runs (its loads then repeat a valid run and store
// nothing): its loads issue while the caller's value stream is in flight,
// and no loop head makes the compiler wait for that stream first.
template <typename T>
__device__ __forceinline__ void stage_runs(const T* __restrict__ v, int2 dsc, int mine, int lane,
                                           T* prod) {
    constexpr int SB = 8;   // runs copied per batch (loads in flight); fits 64 registers
    auto stage_batch = [&](int i0) {
        T tmp[SB];
        int dst[SB];
#pragma unroll
        for (int j = 0; j < SB; ++j) {
            const int i = max(0, min(i0 + j, mine - 1));
            const T* __restrict__ vr = v + __builtin_amdgcn_readlane(dsc.x, i);   // run start
            const int ol = __builtin_amdgcn_readlane(dsc.y, i);
            const int len = ol >> 16;
            tmp[j] = vr[min((unsigned)lane, (unsigned)(len - 1))];
            dst[j] = (i0 + j < mine && lane < len) ? (ol & 0xffff) + lane : -1;
        }
#pragma unroll
        for (int j = 0; j < SB; ++j)
            if (dst[j] >= 0) prod[dst[j]] = tmp[j];
    };
    stage_batch(0);
    for (int i0 = SB; i0 < mine; i0 += SB) stage_batch(i0);
}

// Staged: run table first, then values and slots, then the vector runs
// (copied into prod), then the products (into prod).  nruns > 0.
template <typename T, bool PLAIN>
__device__ __forceinline__ void stage_products(const SpmvArgs<T>& a, int run0, int64_t base, int n,
                                               int nruns, T* prod) {
    constexpr int NT = spmv_threads<T>();
    constexpr int PER = spmv_cap<T>() / NT;
    constexpr int NW = NT / WAVE;
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const int2* __restrict__ runs = reinterpret_cast<const int2*>(a.runs) + run0;
    // runs w, w + NW, ... of this wave; a staged block has at most
    // NT = NW * WAVE runs, so one descriptor per lane
    const int mine = nruns > w ? (nruns - w + NW - 1) / NW : 0;
    const int2 dsc = runs[min(w + NW * lane, nruns - 1)];
    const uint16_t* __restrict__ sl = a.slot + base;
    const T* __restrict__ val = a.val + base;
    int c[PER];
    T av[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        // Guarded (lanes past the block's nonzeros issue nothing): measured
        // faster here than clamped loads, and these guards add no waits
        // between the loads.  Unsigned offsets keep scalar-base addressing.
        const unsigned idx = (unsigned)(tid + k * NT);
        if (idx < (unsigned)n) {
            c[k] = (int)ld_matrix<PLAIN>(sl + idx);
            av[k] = ld_matrix<PLAIN>(val + idx);
        } else {
            c[k] = 0;
            av[k] = T(0);
        }
    }
    stage_runs<T>(a.v, dsc, mine, lane, prod);
    __syncthreads();
    T pr[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) pr[k] = av[k] * prod[c[k]];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = tid + k * NT;
        if (idx < n) prod[idx] = pr[k];
    }
}

// Direct: column ids and values first, then the gathers.  n > 0.
template <typename T, bool PLAIN>
__device__ __forceinline__ void direct_products(const SpmvArgs<T>& a, int64_t base, int n, T* prod) {
    constexpr int NT = spmv_threads<T>();
    constexpr int PER = spmv_cap<T>() / NT;
    const int tid = threadIdx.x;
    const int32_t* __restrict__ ci = a.ci + base;
    const T* __restrict__ val = a.val + base;
    const T* __restrict__ v = a.v;
    int32_t c[PER];
    T av[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const unsigned idx = min((unsigned)(tid + k * NT), (unsigned)(n - 1));
        c[k] = ld_matrix<PLAIN>(ci + idx);
        av[k] = ld_matrix<PLAIN>(val + idx);
    }
    T xv[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) xv[k] = v[c[k]];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = tid + k * NT;
        if (idx < n) prod[idx] = av[k] * xv[k];
    }
}

// Streaming CSR product.  A block of NT = spmv_threads<T>() threads owns a
// run of at most NT whole rows whose nonzeros (at most spmv_cap<T>(): 8 FP64
// values per thread of 1024, 64 KB of LDS, or 16 FP32 values per thread of
// 512, 32 KB) are contiguous, and
// reads where they start from one 32-byte descriptor, so the value stream
// waits on one load only:
//  0. thread t prefetches the row-local operands of row r0 + t and the end
//     of that row (the row sums read the row bounds from LDS);
//  1. every thread issues its eight value loads and eight column loads at
//     once (coalesced, non-temporal) and forms the products in LDS.  With
//     staged gathers the block first copies the vector entries it needs
//     into LDS: the distinct columns of its nonzeros form runs of
//     consecutive ids, a wave copies one run (at most 64 entries) per load,
//     and the run table is read before the values arrive, so the copies
//     overlap the value stream; the nonzeros then carry 16-bit LDS slots in
//     place of column ids.  Without staging each nonzero gathers straight
//     from memory once its column id has arrived.
//  2. groups of L lanes sum the rows from LDS in a fixed order (reads issued
//     ahead of the in-order adds, DPP butterflies);
//  3. thread t finishes row r0 + t (coalesced row-local stores).
// Both forms multiply the same operands and sum in the same order, so they
// give bitwise identical results.  STAGE picks the form at compile time:
// 0 direct everywhere; 1 staged in every block with nonzeros; 2 per block
// (the run count decides).  Forms 0 and 1 keep the other form's code out of
// the kernel, so nothing ahead of the value stream waits on loads.  A row
// longer than the capacity (forms 0 and 2 only) has a block of its own, summed
// straight from memory by the whole block.  STAGE bit 4 (with form 1, FP32
// only) loads the matrix stream with plain instead of non-temporal loads.
// Occupancy target of the streaming product: 8 waves per SIMD (64 VGPRs),
// except the FP32 form that carries both the staged and the direct gathers
// (16 values per thread of each), which needs a few more registers and runs
// at 7 rather than spill to scratch.
template <typename T, int STAGE>
constexpr int stream_waves() { return (sizeof(T) == 4 && (STAGE & 3) == 2) ? 7 : 8; }

template <typename T, int MODE, int L, int STAGE>
__global__ void __launch_bounds__(spmv_threads<T>())
__attribute__((amdgpu_waves_per_eu(stream_waves<T, STAGE>(), 8)))
spmv_stream_kernel(SpmvArgs<T> a) {
    if (stopped(a.stop)) return;
    constexpr int FORM = STAGE & 3;              // 0 direct, 1 staged, 2 per block
    constexpr bool PLAIN = (STAGE & 4) != 0;     // plain matrix-stream loads
    constexpr int CAP = spmv_cap<T>();
    constexpr int NT = spmv_threads<T>();
    __shared__ T prod[CAP];
    __shared__ T rowsum[NT];
    __shared__ int rowoff[NT + 1];
    double* red = reinterpret_cast<double*>(prod);   // reused once products are consumed
    const int tid = threadIdx.x;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const BlockDesc B = a.bdesc[lb];   // one load: no dependent row-pointer reads ahead of the values
    const int64_t r0 = B.r0, base = B.base, cnt = B.n;
    double dot = 0.0, dot2 = 0.0;
    if constexpr (MODE == SPMV_RINIT) {
        if (a.vnz != nullptr && *a.vnz == 0.0) {
            // v = +0 everywhere: the row sums are +0, y = f - 0 = f
            const int nr = cnt > CAP ? 1 : B.nrows;
            if (tid < nr) {
                RowIn<T> in{};
                epilogue_load<T, MODE>(a, r0 + tid, in);
                epilogue_store<T, MODE>(a, r0 + tid, T(0), in, dot, dot2);
            }
            block_sum_to0<NT, n_partials<MODE>()>(red, tid, dot, dot2);
            if (tid == 0) {
                a.partial[lb] = dot;
                a.partial[a.nblk + lb] = dot2;
            }
            return;
        }
    }
    if constexpr (FORM != 1) {
        if (cnt > CAP) {
            // one long row: block-wide strided sum, fixed-order block sum
            const int32_t* __restrict__ ci = a.ci + base;
            const T* __restrict__ val = a.val + base;
            const T* __restrict__ v = a.v;
            RowIn<T> in{};
            if (tid == 0) epilogue_load<T, MODE>(a, r0, in);
            T acc0 = 0, acc1 = 0;
            int64_t i = tid;
            for (; i + NT < cnt; i += 2 * NT) {
                const int32_t c0 = ldnt(ci + i), c1 = ldnt(ci + i + NT);
                const T a0 = ldnt(val + i), a1 = ldnt(val + i + NT);
                acc0 += a0 * v[c0];
                acc1 += a1 * v[c1];
            }
            if (i < cnt) acc0 += ldnt(val + i) * v[ldnt(ci + i)];
            double s = (double)(acc0 + acc1), unused = 0.0;
            block_sum_to0<NT, 1>(red, tid, s, unused);
            const T y = (T)s;
            if (tid == 0) {
                epilogue_store<T, MODE>(a, r0, y, in, dot, dot2);
                if constexpr (has_partials<MODE>()) {
                    a.partial[lb] = dot;
                    if (MODE == SPMV_RINIT) a.partial[a.nblk + lb] = dot2;
                }
            }
            return;
        }
    }
    const int nrows = B.nrows;
    const int n = (int)cnt;
    // 0. row-local operands of this thread's row, and the end of that row
    // (low word of the int64 row pointer: offsets in a block are < 2^12)
    RowIn<T> in{};
    const bool own = tid < nrows;
    uint32_t row_end = 0;
    // (whole waves without rows skip it: a wave-uniform branch, measured 3 %
    // faster on the fine Chebyshev step than every wave loading clamped rows)
    if ((tid / WAVE) * WAVE < nrows) {
        const int64_t row = r0 + min(tid, nrows - 1);
        epilogue_load<T, MODE>(a, row, in);
        row_end = reinterpret_cast<const uint32_t*>(a.rp)[2 * (row + 1)];
    }
    // 1. products into LDS
    if constexpr (FORM == 0) {
        if (n > 0) direct_products<T, PLAIN>(a, base, n, prod);
    } else if constexpr (FORM == 1) {
        if (B.nruns > 0) stage_products<T, PLAIN>(a, B.run0, base, n, B.nruns, prod);   // 0: empty rows only
    } else {
        if (B.nruns > 0)
            stage_products<T, PLAIN>(a, B.run0, base, n, B.nruns, prod);
        else if (n > 0)
            direct_products<T, PLAIN>(a, base, n, prod);
    }
    if (own) rowoff[tid + 1] = (int)(row_end - (uint32_t)base);
    if (tid == 0) rowoff[0] = 0;
    __syncthreads();
    // 2. row sums, L lanes per row
    const int g = tid / L, gl = tid % L;
    for (int rr = g; rr < nrows; rr += NT / L) {
        T acc = lane_row_sum<L>(prod, rowoff[rr], rowoff[rr + 1], gl);
        acc = row_group_sum<L>(acc);
        if (gl == 0) rowsum[rr] = acc;
    }
    __syncthreads();
    // 3. row epilogues
    if (own) epilogue_store<T, MODE>(a, r0 + tid, rowsum[tid], in, dot, dot2);
    if constexpr (has_partials<MODE>()) {
        block_sum_to0<NT, n_partials<MODE>()>(red, tid, dot, dot2);
        if (tid == 0) {
            a.partial[lb] = dot;
            if (MODE == SPMV_RINIT) a.partial[a.nblk + lb] = dot2;
        }
    }
}

// ---------------------------------------------------------------------------
// Grouped form.  Rows whose column lists are identical (in a high-order
// element mesh: the interior, face-interior and edge-interior nodes of one
// element, face or edge) form groups of at most GROUP_ROWS rows; they share
// one list of 16-bit LDS slots, so the slot stream shrinks by the group size.
// A block holds groups of one size G (E entries: the union of its groups'
// lists, group after group) and stores its values as G planes of E values,
// plane i holding row i of every group; its columns are staged in LDS as in
// the CSR form.  Row sums use the CSR form's order and lane split, so both
// forms give the same row results bit for bit (block partial sums of the
// DOT and RINIT epilogues add the rows in another order).
// ---------------------------------------------------------------------------

// Steps 1 and 2 for a block of G-row groups.  Thread t takes entries
// t + k * GROUP_THREADS (k < 8 / G): per entry one slot and G values (one per
// plane), all loads issued before the run copies; products go to LDS plane
// by plane (prod[i * E + e]); then groups of L lanes sum the rows.
template <typename T, int L, int G>
__device__ __forceinline__ void group_block(const SpmvArgs<T>& a, int64_t lb, const GBlock& B, int E,
                                            int R, int nruns, T* prod, T* rowsum) {
    constexpr int KPT = GROUP_CAP / GROUP_THREADS / G;   // entries per thread
    constexpr int NW = GROUP_THREADS / WAVE;
    static_assert(KPT >= 1 && KPT * G <= GROUP_CAP / GROUP_THREADS, "entries per thread");
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    if (nruns > 0) {   // 0 only for blocks of empty rows (E == 0)
        const int2* __restrict__ runs = reinterpret_cast<const int2*>(a.gruns) + a.grun_ptr[lb];
        const int mine = nruns > w ? (nruns - w + NW - 1) / NW : 0;
        const int2 dsc = runs[min(w + NW * lane, nruns - 1)];
        const uint16_t* __restrict__ sl = a.gslot + B.e0;
        const T* __restrict__ val = a.gval + B.v0;
        int c[KPT];
        T av[KPT][G];
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            const unsigned idx = (unsigned)(tid + k * GROUP_THREADS);
            if (idx < (unsigned)E) {
                c[k] = (int)ldnt(sl + idx);
#pragma unroll
                for (int i = 0; i < G; ++i) av[k][i] = ldnt(val + (unsigned)(i * E) + idx);
            } else {
                c[k] = 0;
#pragma unroll
                for (int i = 0; i < G; ++i) av[k][i] = T(0);
            }
        }
        stage_runs<T>(a.v, dsc, mine, lane, prod);
        __syncthreads();
        T pr[KPT][G];
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            const T xv = prod[c[k]];
#pragma unroll
            for (int i = 0; i < G; ++i) pr[k][i] = av[k][i] * xv;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            const int idx = tid + k * GROUP_THREADS;
            if (idx < E) {
#pragma unroll
                for (int i = 0; i < G; ++i) prod[i * E + idx] = pr[k][i];
            }
        }
    }
    __syncthreads();
    const int gi = tid / L, gl = tid % L;
    for (int rr = gi; rr < R; rr += GROUP_THREADS / L) {
        const int q = rr / G, i = rr - q * G;
        const uint32_t gq = a.ggrp[B.q0 + q];
        const int s = i * E + (int)(gq >> 16), e = s + (int)(gq & 0xffffu);
        T acc = lane_row_sum<L>(prod, s, e, gl);
        acc = row_group_sum<L>(acc);
        if (gl == 0) rowsum[rr] = acc;
    }
}

// Product over the grouped form: block lb (XCD-remapped as in the CSR form)
// owns R = G * groups rows listed in grows; thread t finishes row t.
template <typename T, int MODE, int L>
__global__ void __launch_bounds__(GROUP_THREADS) __attribute__((amdgpu_waves_per_eu(8, 8)))
spmv_group_kernel(SpmvArgs<T> a) {
    if (stopped(a.stop)) return;
    __shared__ T prod[GROUP_CAP];
    __shared__ T rowsum[GROUP_THREADS];
    double* red = reinterpret_cast<double*>(prod);
    const int tid = threadIdx.x;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const GBlock B = a.gblk[lb];
    const int E = (int)(a.gblk[lb + 1].e0 - B.e0), R = a.gblk[lb + 1].r0 - B.r0;
    const int nruns = a.grun_ptr[lb + 1] - a.grun_ptr[lb];
    double dot = 0.0, dot2 = 0.0;
    RowIn<T> in{};
    int64_t row = 0;
    if ((tid / WAVE) * WAVE < R) {
        row = a.grows[B.r0 + min(tid, R - 1)];
        epilogue_load<T, MODE>(a, row, in);
    }
    switch (B.g) {
        case 1: group_block<T, L, 1>(a, lb, B, E, R, nruns, prod, rowsum); break;
        case 2: group_block<T, L, 2>(a, lb, B, E, R, nruns, prod, rowsum); break;
        case 3: group_block<T, L, 3>(a, lb, B, E, R, nruns, prod, rowsum); break;
        case 4: group_block<T, L, 4>(a, lb, B, E, R, nruns, prod, rowsum); break;
        case 5: group_block<T, L, 5>(a, lb, B, E, R, nruns, prod, rowsum); break;
        case 6: group_block<T, L, 6>(a, lb, B, E, R, nruns, prod, rowsum); break;
        case 7: group_block<T, L, 7>(a, lb, B, E, R, nruns, prod, rowsum); break;
        default: group_block<T, L, 8>(a, lb, B, E, R, nruns, prod, rowsum); break;
    }
    __syncthreads();
    if (tid < R) epilogue_store<T, MODE>(a, row, rowsum[tid], in, dot, dot2);
    if constexpr (has_partials<MODE>()) {
        block_sum_to0<GROUP_THREADS, n_partials<MODE>()>(red, tid, dot, dot2);
        if (tid == 0) {
            a.partial[lb] = dot;
            if (MODE == SPMV_RINIT) a.partial[a.nblk + lb] = dot2;
        }
    }
}

// ---------------------------------------------------------------------------
// Lean form for small operators (DevCSR::lean): groups of L lanes read a row
// straight from memory (column ids and values, then the vector), with no
// row-block bounds, run tables or LDS staging, so a launch waits on a chain
// three loads deep; the coarse levels (kilobytes to a few MB each) are
// bound by that chain, not by bytes.  Lane gl sums the row's products at
// positions gl, gl + L, ... in order, each product rounded before it is
// added (as the LDS products of the CSR form are), and the L lanes combine
// by the same butterfly: rows equal the CSR form's bit for bit (operators
// with rows longer than spmv_cap<T>() keep the CSR form).
// ---------------------------------------------------------------------------
template <typename T, int MODE, int L>
__global__ void __launch_bounds__(LEAN_THREADS) spmv_lean_kernel(SpmvArgs<T> a) {
    if (stopped(a.stop)) return;
    constexpr int RPB = LEAN_THREADS / L;
    const int tid = threadIdx.x, gl = tid % L;
    const int64_t row = (int64_t)blockIdx.x * RPB + tid / L;
    const bool live = row < a.n;
    const int64_t rr = live ? row : a.n - 1;
    RowIn<T> in{};
    if (gl == 0) epilogue_load<T, MODE>(a, rr, in);
    const int64_t s = a.rp[rr], e = a.rp[rr + 1];
    const int32_t* __restrict__ ci = a.ci;
    const T* __restrict__ val = a.val;
    const T* __restrict__ v = a.v;
    T acc = 0;
    {
#pragma clang fp contract(off)
        int64_t j = s + gl;
        for (; j + 3 * L < e; j += 4 * L) {
            const int32_t c0 = ci[j], c1 = ci[j + L], c2 = ci[j + 2 * L], c3 = ci[j + 3 * L];
            const T a0 = val[j], a1 = val[j + L], a2 = val[j + 2 * L], a3 = val[j + 3 * L];
            const T p0 = a0 * v[c0], p1 = a1 * v[c1], p2 = a2 * v[c2], p3 = a3 * v[c3];
            acc += p0;
            acc += p1;
            acc += p2;
            acc += p3;
        }
        for (; j < e; j += L) {
            const T p = val[j] * v[ci[j]];
            acc += p;
        }
    }
    acc = row_group_sum<L>(acc);
    double dot = 0.0, dot2 = 0.0;
    if (live && gl == 0) epilogue_store<T, MODE>(a, row, acc, in, dot, dot2);
    if constexpr (has_partials<MODE>()) {
        __shared__ double red[2 * LEAN_THREADS / WAVE];
        block_sum_to0<LEAN_THREADS, n_partials<MODE>()>(red, tid, dot, dot2);
        if (tid == 0) {
            a.partial[blockIdx.x] = dot;
            if (MODE == SPMV_RINIT) a.partial[a.nblk + blockIdx.x] = dot2;
        }
    }
}

__global__ void gather_values_kernel(int64_t n, const int64_t* __restrict__ idx, const double* __restrict__ x,
                                     double* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[idx[i]];
}

void launch_gather_values(int64_t n, const int64_t* idx, const double* x, double* y, hipStream_t s) {
    if (n <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    gather_values_kernel<<<g, 256, 0, s>>>(n, idx, x, y);
    GIAMG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Staged-gather tables (setup).  Per row block: a bitmap of the columns its
// nonzeros touch (64-bit words over [cmin, cmax]); a run is a maximal set of
// consecutive set bits inside one word, so it holds at most 64 columns; the
// LDS slot of a column is its rank among the set bits.  Pass 1 counts the
// runs of each block, pass 2 writes the runs and the slot of every nonzero.
// Blocks with more than max_runs runs (one run descriptor per lane of the
// product kernel's block; scattered columns) are left to
// direct gathers, as are blocks spanning more than STAGE_SPAN columns.
// ---------------------------------------------------------------------------
constexpr int STAGE_THREADS = 512;
constexpr int STAGE_WORDS = (int)(STAGE_SPAN / 64);
constexpr int STAGE_WPT = STAGE_WORDS / STAGE_THREADS;
static_assert(STAGE_WORDS % STAGE_THREADS == 0, "bitmap words per thread");

// Exclusive prefix over the block of one int per thread; sum in total.
__device__ int stage_exscan(int v, int* sc, int tid, int& total) {
    sc[tid] = v;
    __syncthreads();
    for (int o = 1; o < STAGE_THREADS; o <<= 1) {
        const int t = tid >= o ? sc[tid - o] : 0;
        __syncthreads();
        sc[tid] += t;
        __syncthreads();
    }
    total = sc[STAGE_THREADS - 1];
    const int incl = sc[tid];
    __syncthreads();
    return incl - v;
}

template <bool FILL>
__global__ void __launch_bounds__(STAGE_THREADS) stage_kernel(const int64_t* __restrict__ rp,
                                                             const int32_t* __restrict__ ci,
                                                             const int64_t* __restrict__ rblk, int cap,
                                                             int max_runs,
                                                             int32_t* counts, const int32_t* run_ptr,
                                                             int32_t* runs, uint16_t* slot) {
    __shared__ unsigned long long bm[STAGE_WORDS];
    __shared__ uint16_t rank_pre[STAGE_WORDS];
    __shared__ uint16_t run_pre[STAGE_WORDS];
    __shared__ int sc[STAGE_THREADS];
    __shared__ int wmin[STAGE_THREADS / WAVE], wmax[STAGE_THREADS / WAVE];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t r0 = rblk[b], r1 = rblk[b + 1];
    const int64_t base = rp[r0];
    const int64_t cnt = rp[r1] - base;
    if (cnt == 0 || cnt > cap) {
        if (!FILL && tid == 0) counts[b] = 0;
        return;
    }
    const int n = (int)cnt;
    const int32_t* c = ci + base;
    int mn = 0x7fffffff, mx = -1;
    for (int i = tid; i < n; i += STAGE_THREADS) {
        const int v = c[i];
        mn = min(mn, v);
        mx = max(mx, v);
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o, WAVE));
        mx = max(mx, __shfl_xor(mx, o, WAVE));
    }
    if (tid % WAVE == 0) {
        wmin[tid / WAVE] = mn;
        wmax[tid / WAVE] = mx;
    }
    __syncthreads();
    mn = wmin[0];
    mx = wmax[0];
    for (int i = 1; i < STAGE_THREADS / WAVE; ++i) {
        mn = min(mn, wmin[i]);
        mx = max(mx, wmax[i]);
    }
    if ((int64_t)mx - mn + 1 > STAGE_SPAN) {       // same decision in every thread
        if (!FILL && tid == 0) counts[b] = 0;
        return;
    }
    const int nw = (int)(((int64_t)mx - mn + 64) >> 6);
    for (int w = tid; w < nw; w += STAGE_THREADS) bm[w] = 0ull;
    __syncthreads();
    for (int i = tid; i < n; i += STAGE_THREADS) {
        const int o = c[i] - mn;
        atomicOr(&bm[o >> 6], 1ull << (o & 63));
    }
    __syncthreads();
    const int w0 = tid * STAGE_WPT, w1 = min(nw, w0 + STAGE_WPT);
    int pc = 0, rc = 0;
    for (int w = w0; w < w1; ++w) {
        const unsigned long long x = bm[w];
        pc += __popcll(x);
        rc += __popcll(x & ~(x << 1));
    }
    int tot_runs = 0, tot_cols = 0;
    int rex = stage_exscan(rc, sc, tid, tot_runs);
    if (!FILL) {
        if (tid == 0) counts[b] = tot_runs <= max_runs ? tot_runs : 0;
        return;
    }
    if (tot_runs > max_runs) return;   // scattered columns: direct gathers
    int uex = stage_exscan(pc, sc, tid, tot_cols);
    for (int w = w0; w < w1; ++w) {
        const unsigned long long x = bm[w];
        rank_pre[w] = (uint16_t)uex;
        run_pre[w] = (uint16_t)rex;
        uex += __popcll(x);
        rex += __popcll(x & ~(x << 1));
    }
    __syncthreads();
    int32_t* out = runs + 2 * (int64_t)run_ptr[b];
    for (int w = w0; w < w1; ++w) {
        const unsigned long long x = bm[w];
        unsigned long long st = x & ~(x << 1);
        int ri = run_pre[w];
        while (st) {
            const int pos = __ffsll((long long)st) - 1;
            const unsigned long long rest = ~(x >> pos);
            const int len = rest ? __ffsll((long long)rest) - 1 : 64 - pos;
            const int rank = rank_pre[w] + __popcll(x & ((1ull << pos) - 1ull));
            out[2 * ri] = mn + w * 64 + pos;
            out[2 * ri + 1] = rank | (len << 16);
            ++ri;
            st &= st - 1ull;
        }
    }
    for (int i = tid; i < n; i += STAGE_THREADS) {
        const int o = c[i] - mn;
        const int w = o >> 6, pos = o & 63;
        slot[base + i] = (uint16_t)(rank_pre[w] + __popcll(bm[w] & ((1ull << pos) - 1ull)));
    }
}

void build_staging(const DevCSR& d, RowBlocks& B, const std::vector<int64_t>& rp, hipStream_t s) {
    B.release_staging();
    if (B.nblk <= 0 || d.nnz <= 0) return;
    GIAMG_REQUIRE(B.nblk < (int64_t(1) << 31), "too many row blocks");
    DevBuf<int32_t> counts(B.nblk);
    GIAMG_REQUIRE(B.threads > 0 && B.threads % WAVE == 0, "row blocks without a thread count");
    stage_kernel<false><<<(unsigned)B.nblk, STAGE_THREADS, 0, s>>>(d.rp.get(), d.ci.get(), B.rblk.get(), B.cap,
                                                                  B.threads, counts.get(), nullptr, nullptr,
                                                                  nullptr);
    GIAMG_HIP(hipGetLastError());
    std::vector<int32_t> hc(B.nblk);
    std::vector<int64_t> hb(B.nblk + 1);
    GIAMG_HIP(hipMemcpyAsync(hc.data(), counts.get(), B.nblk * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipMemcpyAsync(hb.data(), B.rblk.get(), (B.nblk + 1) * sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> ptr(B.nblk + 1, 0);
    int64_t total = 0, staged = 0;
    for (int64_t b = 0; b < B.nblk; ++b) {
        ptr[b] = (int32_t)total;
        total += hc[b];
        if (hc[b] > 0) staged += rp[hb[b + 1]] - rp[hb[b]];
        if (total >= (int64_t(1) << 31)) return;   // tables too large: direct gathers throughout
    }
    ptr[B.nblk] = (int32_t)total;
    if (total == 0) return;
    B.run_ptr.alloc(B.nblk + 1);
    B.runs.alloc(2 * total);
    B.slot.alloc(d.nnz);
    GIAMG_HIP(hipMemcpyAsync(B.run_ptr.get(), ptr.data(), ptr.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s));
    stage_kernel<true><<<(unsigned)B.nblk, STAGE_THREADS, 0, s>>>(d.rp.get(), d.ci.get(), B.rblk.get(), B.cap,
                                                                 B.threads, nullptr, B.run_ptr.get(),
                                                                 B.runs.get(), B.slot.get());
    GIAMG_HIP(hipGetLastError());
    GIAMG_HIP(hipStreamSynchronize(s));
    B.nruns = total;
    B.nnz_staged = staged;
}

template <typename T, int MODE, int L, int STAGE>
void launch_spmv_kernel(const SpmvArgs<T>& a, hipStream_t s) {
    const dim3 grid((unsigned)a.nblk), block(spmv_threads<T>());
    if (a.ev_start != nullptr)   // timing: the dispatch records the events itself
        hipExtLaunchKernelGGL(spmv_stream_kernel<T, MODE, L, STAGE>, grid, block, 0, s, a.ev_start,
                              a.ev_stop, 0, a);
    else
        spmv_stream_kernel<T, MODE, L, STAGE><<<grid, block, 0, s>>>(a);
}

template <typename T, int MODE, int L>
void launch_group_kernel(const SpmvArgs<T>& a, hipStream_t s) {
    const dim3 grid((unsigned)a.nblk), block(GROUP_THREADS);
    if (a.ev_start != nullptr)
        hipExtLaunchKernelGGL(spmv_group_kernel<T, MODE, L>, grid, block, 0, s, a.ev_start, a.ev_stop, 0, a);
    else
        spmv_group_kernel<T, MODE, L><<<grid, block, 0, s>>>(a);
}

template <typename T, int MODE, int STAGE>
void launch_spmv_form(const SpmvArgs<T>& a, hipStream_t s) {
    switch (a.lanes) {
        case 16: launch_spmv_kernel<T, MODE, 16, STAGE>(a, s); break;
        case 4: launch_spmv_kernel<T, MODE, 4, STAGE>(a, s); break;
        case 1: launch_spmv_kernel<T, MODE, 1, STAGE>(a, s); break;
        default: throw Error(GIAMG_EINVAL, "unsupported reduction width");
    }
}

template <typename T, int MODE, int L>
void launch_lean_kernel(const SpmvArgs<T>& a, hipStream_t s) {
    const dim3 grid((unsigned)a.nblk), block(LEAN_THREADS);
    if (a.ev_start != nullptr)
        hipExtLaunchKernelGGL(spmv_lean_kernel<T, MODE, L>, grid, block, 0, s, a.ev_start, a.ev_stop, 0, a);
    else
        spmv_lean_kernel<T, MODE, L><<<grid, block, 0, s>>>(a);
}

template <typename T, int MODE>
void launch_spmv_mode(const SpmvArgs<T>& a, hipStream_t s) {
    if (a.lean) {
        switch (a.lanes) {
            case 16: launch_lean_kernel<T, MODE, 16>(a, s); break;
            case 4: launch_lean_kernel<T, MODE, 4>(a, s); break;
            case 1: launch_lean_kernel<T, MODE, 1>(a, s); break;
            default: throw Error(GIAMG_EINVAL, "unsupported reduction width");
        }
    } else if (a.gblk != nullptr) {
        switch (a.lanes) {
            case 16: launch_group_kernel<T, MODE, 16>(a, s); break;
            case 4: launch_group_kernel<T, MODE, 4>(a, s); break;
            case 1: launch_group_kernel<T, MODE, 1>(a, s); break;
            default: throw Error(GIAMG_EINVAL, "unsupported reduction width");
        }
    } else if (a.run_ptr == nullptr) {
        launch_spmv_form<T, MODE, 0>(a, s);
    } else if (a.nnz_staged == a.nnz) {
        if constexpr (sizeof(T) == sizeof(float)) {
            if (a.nnz >= FP32_PLAIN_MIN_NNZ) {
                launch_spmv_form<T, MODE, 1 | 4>(a, s);
                return;
            }
        }
        launch_spmv_form<T, MODE, 1>(a, s);
    } else {
        launch_spmv_form<T, MODE, 2>(a, s);
    }
}

template <typename T>
void launch_spmv(int mode, const SpmvArgs<T>& args, hipStream_t s) {
    SpmvArgs<T> a = args;
    if (a.stop == nullptr) a.stop = g_stop;
    if (a.n <= 0 || a.nblk <= 0) return;
    if (!a.lean && a.gblk == nullptr) {
        if (a.rblk == nullptr || a.bdesc == nullptr) throw Error(GIAMG_EINVAL, "operator without row blocks");
        // the kernel's LDS arrays hold spmv_cap<T>() products and spmv_threads<T>() rows
        if (a.block_cap != spmv_cap<T>() || a.block_threads != spmv_threads<T>())
            throw Error(GIAMG_EINVAL, "row blocks built for another block shape");
    }
    switch (mode) {
        case SPMV_PLAIN: launch_spmv_mode<T, SPMV_PLAIN>(a, s); break;
        case SPMV_RESID: launch_spmv_mode<T, SPMV_RESID>(a, s); break;
        case SPMV_ADD: launch_spmv_mode<T, SPMV_ADD>(a, s); break;
        case SPMV_CHEB_INIT: launch_spmv_mode<T, SPMV_CHEB_INIT>(a, s); break;
        case SPMV_CHEB_STEP: launch_spmv_mode<T, SPMV_CHEB_STEP>(a, s); break;
        case SPMV_JACOBI: launch_spmv_mode<T, SPMV_JACOBI>(a, s); break;
        case SPMV_DOT: launch_spmv_mode<T, SPMV_DOT>(a, s); break;
        case SPMV_DINV: launch_spmv_mode<T, SPMV_DINV>(a, s); break;
        case SPMV_RINIT: launch_spmv_mode<T, SPMV_RINIT>(a, s); break;
        case SPMV_RCHEB0: launch_spmv_mode<T, SPMV_RCHEB0>(a, s); break;
        default: throw Error(GIAMG_EINVAL, "unknown product mode");
    }
    GIAMG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Attainable read bandwidth: a streaming read shaped like the products'
// value stream -- each block of 512 threads reads one contiguous 64 KB chunk
// with all eight 16-byte non-temporal loads per thread issued at once, blocks
// remapped so every XCD streams a contiguous range -- over a zeroed buffer,
// with a store that only a nonzero sum would make.
// ---------------------------------------------------------------------------
typedef double double2_v __attribute__((ext_vector_type(2)));
constexpr int RS_THREADS = 512, RS_LOADS = 8;

__global__ void __launch_bounds__(RS_THREADS) read_stream_kernel(const double2_v* __restrict__ p, int64_t n2,
                                                                 double* __restrict__ out) {
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t base = lb * (int64_t)(RS_THREADS * RS_LOADS);
    double2_v v[RS_LOADS];
#pragma unroll
    for (int k = 0; k < RS_LOADS; ++k) {
        const int64_t i = min(base + k * RS_THREADS + threadIdx.x, n2 - 1);
        v[k] = ldnt(p + i);
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RS_LOADS; ++k) acc += v[k].x + v[k].y;
    // the buffer holds zeros: the store never happens, but the compiler
    // cannot drop the loads, and no reduction lengthens the block
    if (acc != 0.0) out[lb] = acc;
}

void read_bandwidth(int64_t bytes, int reps, double* gbs) {
    GIAMG_REQUIRE(bytes >= (int64_t(1) << 20), "bytes must be at least 1 MiB");
    GIAMG_REQUIRE(reps >= 1 && reps <= 1000, "reps must be in [1, 1000]");
    const int64_t n2 = bytes / 16;
    const unsigned grid = (unsigned)((n2 + RS_THREADS * RS_LOADS - 1) / (RS_THREADS * RS_LOADS));
    DevBuf<double2_v> buf(n2);
    DevBuf<double> out(grid);
    hipStream_t s = nullptr;
    GIAMG_HIP(hipMemsetAsync(buf.get(), 0, n2 * 16, s));
    std::vector<hipEvent_t> ev(2 * (size_t)reps + 2, nullptr);
    std::vector<double> rate;
    try {
        for (auto& e : ev) GIAMG_HIP(hipEventCreate(&e));
        // one untimed launch, then the timed ones
        for (int i = 0; i <= reps; ++i) {
            hipExtLaunchKernelGGL(read_stream_kernel, dim3(grid), dim3(RS_THREADS), 0, s, ev[2 * i],
                                  ev[2 * i + 1], 0, buf.get(), n2, out.get());
            GIAMG_HIP(hipGetLastError());
        }
        GIAMG_HIP(hipEventSynchronize(ev[2 * reps + 1]));
        for (int i = 1; i <= reps; ++i) {
            float t = 0.0f;
            GIAMG_HIP(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
            rate.push_back((double)n2 * 16.0 / (t * 1e-3) / 1e9);
        }
    } catch (...) {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        throw;
    }
    for (auto e : ev) (void)hipEventDestroy(e);
    std::sort(rate.begin(), rate.end());
    *gbs = rate[rate.size() / 2];
}

template void launch_spmv<double>(int, const SpmvArgs<double>&, hipStream_t);
template void launch_spmv<float>(int, const SpmvArgs<float>&, hipStream_t);

// ---------------------------------------------------------------------------
// row-local vector kernels
// ---------------------------------------------------------------------------
static inline unsigned vgrid(int64_t n) {
    int64_t b = (n + VEC_THREADS - 1) / VEC_THREADS;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

template <typename T>
__global__ void cheb_init0_kernel(int64_t n, const T* __restrict__ f, const T* __restrict__ dinv,
                                  T* __restrict__ r, T* __restrict__ d, T* __restrict__ x,
                                  T inv_theta, int write_x, const int* stop) {
    if (stopped(stop)) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T res = dinv[i] * f[i];
        const T dd = res * inv_theta;
        r[i] = res;
        d[i] = dd;
        if (write_x) x[i] = dd;
    }
}
template <typename T>
void launch_cheb_init0(int64_t n, const T* f, const T* dinv, T* r, T* d, T* x, T inv_theta,
                       bool write_x, hipStream_t s) {
    if (n <= 0) return;
    cheb_init0_kernel<T><<<vgrid(n), VEC_THREADS, 0, s>>>(n, f, dinv, r, d, x, inv_theta, write_x, g_stop);
    GIAMG_HIP(hipGetLastError());
}
template void launch_cheb_init0<double>(int64_t, const double*, const double*, double*, double*,
                                        double*, double, bool, hipStream_t);
template void launch_cheb_init0<float>(int64_t, const float*, const float*, float*, float*, float*,
                                       float, bool, hipStream_t);

template <typename T>
__global__ void jacobi0_kernel(int64_t n, const T* __restrict__ f, const T* __restrict__ dinv,
                               T* __restrict__ x, T omega, const int* stop) {
    if (stopped(stop)) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = omega * dinv[i] * f[i];
}
template <typename T>
void launch_jacobi0(int64_t n, const T* f, const T* dinv, T* x, T omega, hipStream_t s) {
    if (n <= 0) return;
    jacobi0_kernel<T><<<vgrid(n), VEC_THREADS, 0, s>>>(n, f, dinv, x, omega, g_stop);
    GIAMG_HIP(hipGetLastError());
}
template void launch_jacobi0<double>(int64_t, const double*, const double*, double*, double,
                                     hipStream_t);
template void launch_jacobi0<float>(int64_t, const float*, const float*, float*, float, hipStream_t);

template <typename T>
__global__ void copy_kernel(int64_t n, const T* __restrict__ a, T* __restrict__ b, const int* stop) {
    if (stopped(stop)) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}
template <typename T>
void launch_copy(int64_t n, const T* a, T* b, hipStream_t s) {
    if (n <= 0) return;
    copy_kernel<T><<<vgrid(n), VEC_THREADS, 0, s>>>(n, a, b, g_stop);
    GIAMG_HIP(hipGetLastError());
}
template void launch_copy<double>(int64_t, const double*, double*, hipStream_t);
template void launch_copy<float>(int64_t, const float*, float*, hipStream_t);

template <typename T>
__global__ void add_kernel(int64_t n, const T* __restrict__ a, T* __restrict__ b, const int* stop) {
    if (stopped(stop)) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] += a[i];
}
template <typename T>
void launch_add(int64_t n, const T* a, T* b, hipStream_t s) {
    if (n <= 0) return;
    add_kernel<T><<<vgrid(n), VEC_THREADS, 0, s>>>(n, a, b, g_stop);
    GIAMG_HIP(hipGetLastError());
}
template void launch_add<double>(int64_t, const double*, double*, hipStream_t);
template void launch_add<float>(int64_t, const float*, float*, hipStream_t);

template <typename Tin, typename Tout>
__global__ void convert_kernel(int64_t n, const Tin* __restrict__ a, Tout* __restrict__ b,
                               const int* stop) {
    if (stopped(stop)) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (Tout)a[i];
}
template <typename Tin, typename Tout>
void launch_convert(int64_t n, const Tin* a, Tout* b, hipStream_t s) {
    if (n <= 0) return;
    convert_kernel<Tin, Tout><<<vgrid(n), VEC_THREADS, 0, s>>>(n, a, b, g_stop);
    GIAMG_HIP(hipGetLastError());
}
template void launch_convert<double, float>(int64_t, const double*, float*, hipStream_t);
template void launch_convert<float, double>(int64_t, const float*, double*, hipStream_t);

__global__ void fill_kernel(int64_t n, double v, double* __restrict__ x) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}
void launch_fill(int64_t n, double v, double* x, hipStream_t s) {
    if (n <= 0) return;
    fill_kernel<<<vgrid(n), VEC_THREADS, 0, s>>>(n, v, x);
    GIAMG_HIP(hipGetLastError());
}

__global__ void mul_kernel(int64_t n, const double* __restrict__ d, const double* __restrict__ x,
                           double* __restrict__ y, const int* stop) {
    if (stopped(stop)) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = d[i] * x[i];
}
void launch_mul(int64_t n, const double* d, const double* x, double* y, hipStream_t s) {
    if (n <= 0) return;
    mul_kernel<<<vgrid(n), VEC_THREADS, 0, s>>>(n, d, x, y, g_stop);
    GIAMG_HIP(hipGetLastError());
}

__global__ void scale_kernel(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i];
}
void launch_scale(int64_t n, double a, const double* x, double* y, hipStream_t s) {
    if (n <= 0) return;
    scale_kernel<<<vgrid(n), VEC_THREADS, 0, s>>>(n, a, x, y);
    GIAMG_HIP(hipGetLastError());
}

// Coarsest level: x = inv f with the dense symmetric inverse, one wavefront
// per row, FP64 accumulation whatever the vector type.
template <typename T>
__global__ void __launch_bounds__(256) coarse_kernel(int64_t n, const double* __restrict__ inv,
                                                     const T* __restrict__ f, T* __restrict__ x,
                                                     const int* stop) {
    if (stopped(stop)) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t row = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (row >= n) return;
    double acc = 0.0;
    const double* a = inv + row * n;
    for (int64_t j = lane; j < n; j += WAVE) acc += a[j] * (double)f[j];
    acc = wave_sum(acc);
    if (lane == 0) x[row] = (T)acc;
}
template <typename T>
void launch_coarse_apply(int64_t n, const double* inv, const T* f, T* x, hipStream_t s) {
    if (n <= 0) return;
    coarse_kernel<T><<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, inv, f, x, g_stop);
    GIAMG_HIP(hipGetLastError());
}
template void launch_coarse_apply<double>(int64_t, const double*, const double*, double*,
                                          hipStream_t);
template void launch_coarse_apply<float>(int64_t, const double*, const float*, float*, hipStream_t);

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
int64_t vec_blocks(int64_t n) {
    int64_t b = (n + 4 * VEC_THREADS - 1) / (4 * VEC_THREADS);
    return std::max<int64_t>(1, std::min<int64_t>(b, VEC_MAX_BLOCKS));
}

// Fixed-order block sum returned to every thread: a butterfly inside each
// wave, then the waves' sums in wave order (sh holds NT / WAVE doubles; the
// trailing barrier lets the caller reuse it at once).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    constexpr int NW = NT / WAVE;
    v = wave_butterfly(v);
    if (threadIdx.x % WAVE == 0) sh[threadIdx.x / WAVE] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// b FP64, or the FP32 output of a mixed-precision V-cycle widened exactly
// flag = 1 when some entry of x has a nonzero bit pattern (-0 counts as
// nonzero); the flag starts at 0 and is only ever set to 1.
__global__ void __launch_bounds__(VEC_THREADS) nonzero_flag_kernel(int64_t n, const double* __restrict__ x,
                                                                   double* __restrict__ flag) {
    bool nz = false;
    for (int64_t i = blockIdx.x * (int64_t)VEC_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * VEC_THREADS)
        nz = nz || __double_as_longlong(x[i]) != 0;
    if (__ballot(nz) != 0 && threadIdx.x % WAVE == 0) *flag = 1.0;
}

void launch_nonzero_flag(int64_t n, const double* x, double* flag, hipStream_t s) {
    if (n <= 0) return;
    nonzero_flag_kernel<<<(unsigned)vec_blocks(n), VEC_THREADS, 0, s>>>(n, x, flag);
    GIAMG_HIP(hipGetLastError());
}

template <typename TB>
__global__ void __launch_bounds__(VEC_THREADS) dot_partial_kernel(int64_t n, const double* __restrict__ a,
                                                                  const TB* __restrict__ b,
                                                                  double* __restrict__ partial,
                                                                  const int* stop) {
    if (stopped(stop)) return;
    __shared__ double sh[VEC_THREADS];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VEC_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VEC_THREADS)
        s += a[i] * (double)b[i];
    s = block_sum<VEC_THREADS>(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
template <typename TB>
void launch_dot_partial(int64_t n, const double* a, const TB* b, double* partial, hipStream_t s) {
    dot_partial_kernel<TB><<<(unsigned)vec_blocks(n), VEC_THREADS, 0, s>>>(n, a, b, partial, g_stop);
    GIAMG_HIP(hipGetLastError());
}
template void launch_dot_partial<double>(int64_t, const double*, const double*, double*, hipStream_t);
template void launch_dot_partial<float>(int64_t, const double*, const float*, double*, hipStream_t);

template <typename TB>
__global__ void __launch_bounds__(VEC_THREADS) dot2_partial_kernel(int64_t n, const double* __restrict__ a,
                                                                   const TB* __restrict__ b,
                                                                   const double* __restrict__ c,
                                                                   double* __restrict__ partial,
                                                                   const int* stop) {
    if (stopped(stop)) return;
    __shared__ double sh[VEC_THREADS];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VEC_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VEC_THREADS) {
        const double bi = (double)b[i];
        s0 += a[i] * bi;
        s1 += c[i] * bi;
    }
    s0 = block_sum<VEC_THREADS>(s0, sh);
    s1 = block_sum<VEC_THREADS>(s1, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s0;
        partial[gridDim.x + blockIdx.x] = s1;
    }
}
template <typename TB>
void launch_dot2_partial(int64_t n, const double* a, const TB* b, const double* c, double* partial,
                         hipStream_t s) {
    dot2_partial_kernel<TB><<<(unsigned)vec_blocks(n), VEC_THREADS, 0, s>>>(n, a, b, c, partial, g_stop);
    GIAMG_HIP(hipGetLastError());
}
template void launch_dot2_partial<double>(int64_t, const double*, const double*, const double*, double*,
                                          hipStream_t);
template void launch_dot2_partial<float>(int64_t, const double*, const float*, const double*, double*,
                                         hipStream_t);

// out[c] = sum_{i<m} partial[c*stride + i] for c < ncomp, fixed order; then
// thread 0 applies the CG scalar update `fin` to the scalar block.
// FIN_CONV closes an iteration: ctl[0] (the stop flag) becomes 2 on a
// breakdown flagged in it (the iteration is not counted); otherwise ctl[1]
// counts it and ctl[0] becomes 1 when ||r|| / ||b|| < tol (the operations
// the host would use), 2 on a non-finite residual, 3 when ctl[1] reaches
// ctl[2].
__device__ void cg_finish(int fin, double* scal, int* ctl) {
    if (fin == FIN_CONV) {
        if (scal[S_FLAG] != 0.0) {   // breakdown in this iteration: not counted
            ctl[0] = 2;
            return;
        }
        const int k = ctl[1] + 1;
        ctl[1] = k;
        const double relres = sqrt(scal[S_RR]) / sqrt(scal[S_BB]);
        if (!isfinite(relres))
            ctl[0] = 2;
        else if (relres < scal[S_TOL])
            ctl[0] = 1;
        else if (k >= ctl[2])
            ctl[0] = 3;
        return;
    }
    if (fin == FIN_ALPHA) {
        const double pq = scal[S_PQ];
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(scal[S_RZ])) {
            scal[S_FLAG] = 1.0;
            scal[S_ALPHA] = 0.0;
        } else {
            scal[S_ALPHA] = scal[S_RZ] / pq;
        }
    } else if (fin == FIN_BETA_FIRST || fin == FIN_BETA || fin == FIN_BETA_FLEX) {
        const double rzn = scal[S_RZNEW];
        if (fin == FIN_BETA_FIRST)
            scal[S_BETA] = 0.0;
        else if (fin == FIN_BETA_FLEX)
            scal[S_BETA] = (rzn - scal[S_ZROLD]) / scal[S_RZ];
        else
            scal[S_BETA] = rzn / scal[S_RZ];
        if (!isfinite(rzn)) scal[S_FLAG] = 1.0;
        scal[S_RZ] = rzn;
    }
}

__global__ void __launch_bounds__(RED_THREADS) reduce_kernel(int64_t m, const double* __restrict__ partial,
                                                             int64_t stride, int ncomp,
                                                             double* out, int fin,
                                                             double* scal,   // out may lie inside scal
                                                             int* ctl, const int* stop) {
    if (stopped(stop)) return;
    __shared__ double sh[RED_THREADS];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int64_t i = threadIdx.x; i < m; i += RED_THREADS) s += partial[c * stride + i];
        s = block_sum<RED_THREADS>(s, sh);
        if (threadIdx.x == 0) out[c] = s;
    }
    if (fin != FIN_NONE && threadIdx.x == 0) {
        __threadfence_block();
        cg_finish(fin, scal, ctl);
    }
}
void launch_reduce(int64_t m, const double* partial, int64_t stride, int ncomp, double* out,
                   hipStream_t s, int fin, double* scal, int* ctl) {
    if (fin == FIN_CONV && ctl == nullptr) throw Error(GIAMG_EINVAL, "convergence test without control block");
    reduce_kernel<<<1, RED_THREADS, 0, s>>>(m, partial, stride, ncomp, out, fin, scal, ctl, g_stop);
    GIAMG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// CG kernels
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(VEC_THREADS) pcg_update_kernel(int64_t n, double* __restrict__ x,
                                                                 double* __restrict__ r,
                                                                 double* __restrict__ rold,
                                                                 const double* __restrict__ p,
                                                                 const double* __restrict__ q,
                                                                 const double* __restrict__ scal,
                                                                 double* __restrict__ partial,
                                                                 const int* stop) {
    if (stopped(stop)) return;
    __shared__ double sh[VEC_THREADS];
    const double alpha = scal[S_ALPHA];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VEC_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VEC_THREADS) {
        x[i] += alpha * p[i];
        const double ri = r[i];
        if (rold) rold[i] = ri;
        const double rn = ri - alpha * q[i];
        r[i] = rn;
        s += rn * rn;
    }
    s = block_sum<VEC_THREADS>(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
void launch_pcg_update(int64_t n, double* x, double* r, double* rold, const double* p,
                       const double* q, const double* scal, double* partial, hipStream_t s) {
    pcg_update_kernel<<<(unsigned)vec_blocks(n), VEC_THREADS, 0, s>>>(n, x, r, rold, p, q, scal, partial,
                                                                    g_stop);
    GIAMG_HIP(hipGetLastError());
}

// The flexible-CG update of a mixed-precision solve: also r_new rounded to
// FP32 (f32, the V-cycle input), and with dinv32 set the fine level's FP32
// zero-start Chebyshev init (cr = dinv32 f32, cd = cr inv_theta: the
// operations of cheb_init0_kernel<float>, so the same bits).
__global__ void __launch_bounds__(VEC_THREADS) pcg_update_mixed_kernel(
    int64_t n, double* __restrict__ x, double* __restrict__ r, double* __restrict__ rold,
    const double* __restrict__ p, const double* __restrict__ q, const double* __restrict__ scal,
    double* __restrict__ partial, float* __restrict__ f32, const float* __restrict__ dinv32,
    float* __restrict__ cr, float* __restrict__ cd, float inv_theta, const int* stop) {
    if (stopped(stop)) return;
    __shared__ double sh[VEC_THREADS];
    const double alpha = scal[S_ALPHA];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VEC_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VEC_THREADS) {
        x[i] += alpha * p[i];
        const double ri = r[i];
        rold[i] = ri;
        const double rn = ri - alpha * q[i];
        r[i] = rn;
        s += rn * rn;
        const float fi = (float)rn;
        f32[i] = fi;
        if (dinv32) {
            const float res = dinv32[i] * fi;
            cr[i] = res;
            cd[i] = res * inv_theta;
        }
    }
    s = block_sum<VEC_THREADS>(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
void launch_pcg_update_mixed(int64_t n, double* x, double* r, double* rold, const double* p,
                             const double* q, const double* scal, double* partial, float* f32,
                             const float* dinv32, float* cr, float* cd, float inv_theta, hipStream_t s) {
    pcg_update_mixed_kernel<<<(unsigned)vec_blocks(n), VEC_THREADS, 0, s>>>(
        n, x, r, rold, p, q, scal, partial, f32, dinv32, cr, cd, inv_theta, g_stop);
    GIAMG_HIP(hipGetLastError());
}

__global__ void __launch_bounds__(VEC_THREADS) pcg_update_cheb0_kernel(
    int64_t n, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, const double* __restrict__ scal, double* __restrict__ partial,
    const double* __restrict__ dinv, double* __restrict__ cr, double* __restrict__ cd, double inv_theta,
    const int* stop) {
    if (stopped(stop)) return;
    __shared__ double sh[VEC_THREADS];
    const double alpha = scal[S_ALPHA];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VEC_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VEC_THREADS) {
        x[i] += alpha * p[i];
        const double rn = r[i] - alpha * q[i];
        r[i] = rn;
        s += rn * rn;
        const double res = dinv[i] * rn;   // the operations of cheb_init0_kernel
        cr[i] = res;
        cd[i] = res * inv_theta;
    }
    s = block_sum<VEC_THREADS>(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
void launch_pcg_update_cheb0(int64_t n, double* x, double* r, const double* p, const double* q,
                             const double* scal, double* partial, const double* dinv, double* cr,
                             double* cd, double inv_theta, hipStream_t s) {
    pcg_update_cheb0_kernel<<<(unsigned)vec_blocks(n), VEC_THREADS, 0, s>>>(n, x, r, p, q, scal, partial,
                                                                          dinv, cr, cd, inv_theta, g_stop);
    GIAMG_HIP(hipGetLastError());
}

template <typename TZ>
__global__ void pcg_direction_kernel(int64_t n, const TZ* __restrict__ z, double* __restrict__ p,
                                     const double* __restrict__ scal, const int* stop) {
    if (stopped(stop)) return;
    const double beta = scal[S_BETA];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (double)z[i] + beta * p[i];
}
template <typename TZ>
void launch_pcg_direction(int64_t n, const TZ* z, double* p, const double* scal, hipStream_t s) {
    pcg_direction_kernel<TZ><<<vgrid(n), VEC_THREADS, 0, s>>>(n, z, p, scal, g_stop);
    GIAMG_HIP(hipGetLastError());
}
template void launch_pcg_direction<double>(int64_t, const double*, double*, const double*, hipStream_t);
template void launch_pcg_direction<float>(int64_t, const float*, double*, const double*, hipStream_t);

// power-iteration start vector v_i = 2 u(h(i)) - 1, h = SplitMix64 stream of
// seed 0, u = top 53 bits scaled to [0, 1)
__global__ void power_start_kernel(int64_t n, double* v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v[i] = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
    }
}
void launch_power_start(int64_t n, double* v, hipStream_t s) {
    if (n <= 0) return;
    power_start_kernel<<<vgrid(n), VEC_THREADS, 0, s>>>(n, v);
    GIAMG_HIP(hipGetLastError());
}

}  // namespace giamg
