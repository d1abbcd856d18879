// Device sparse matrix-matrix product C = A B for the Galerkin coarse
// operators R (A P) (Section 2.1: coarse operators precomputed at setup).
//
// Row-wise (Gustavson) product, one wavefront per row of A, in four passes:
//  1. count the distinct columns of each row in an LDS hash table;
//  2. exclusive scan of the counts into row pointers;
//  3. refill the table, compact it and rank-sort the keys: ascending columns;
//  4. numeric pass: lanes split into groups, group g takes the entries of
//     A's row with index = g mod G in order, its lanes take distinct entries
//     of the matching row of B and accumulate into the group's own LDS
//     accumulator at the position found by binary search; the G accumulators
//     are added in group order.  No floating-point atomics: the result is
//     bitwise reproducible.
// The structure is the full symbolic product (no value-based pruning).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>

#include "internal.h"

namespace giamg {

constexpr int SG_WAVE = 64;
constexpr int SG_HASH = 4096;            // LDS hash slots per row
constexpr int SG_MAX_ROW = SG_HASH / 2;  // load factor <= 1/2

__device__ __forceinline__ uint32_t sg_hash(int32_t k) {
    return ((uint32_t)k * 2654435761u) & (SG_HASH - 1);
}

// Insert every column of row i of A B into the table; returns nothing, the
// count and overflow are accumulated in LDS.
__device__ __forceinline__ void sg_insert_row(const int64_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                              const int64_t* __restrict__ brp, const int32_t* __restrict__ bci,
                                              int64_t i, int lane, int32_t* keys, int* count, int* overflow) {
    for (int64_t s = arp[i] + lane; s < arp[i + 1]; s += SG_WAVE) {
        const int32_t k = aci[s];
        for (int64_t t = brp[k]; t < brp[k + 1]; ++t) {
            const int32_t j = bci[t];
            uint32_t h = sg_hash(j);
            int probes = 0;
            while (true) {
                const int32_t old = atomicCAS(&keys[h], -1, j);
                if (old == -1) {
                    atomicAdd(count, 1);
                    break;
                }
                if (old == j) break;
                h = (h + 1) & (SG_HASH - 1);
                if (++probes >= SG_HASH) {
                    atomicOr(overflow, 1);
                    break;
                }
            }
        }
    }
}

__global__ void __launch_bounds__(SG_WAVE) sg_count_kernel(int64_t n, const int64_t* __restrict__ arp,
                                                           const int32_t* __restrict__ aci,
                                                           const int64_t* __restrict__ brp,
                                                           const int32_t* __restrict__ bci,
                                                           int32_t* __restrict__ counts) {
    __shared__ int32_t keys[SG_HASH];
    __shared__ int count, overflow;
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    for (int h = lane; h < SG_HASH; h += SG_WAVE) keys[h] = -1;
    if (lane == 0) { count = 0; overflow = 0; }
    __syncthreads();
    sg_insert_row(arp, aci, brp, bci, i, lane, keys, &count, &overflow);
    __syncthreads();
    if (lane == 0) counts[i] = (overflow || count > SG_MAX_ROW) ? -1 : count;
}

__global__ void __launch_bounds__(SG_WAVE) sg_fill_kernel(int64_t n, const int64_t* __restrict__ arp,
                                                          const int32_t* __restrict__ aci,
                                                          const int64_t* __restrict__ brp,
                                                          const int32_t* __restrict__ bci,
                                                          const int64_t* __restrict__ crp,
                                                          int32_t* __restrict__ cci) {
    __shared__ int32_t keys[SG_HASH];
    __shared__ int32_t packed[SG_MAX_ROW];
    __shared__ int count, overflow, npack;
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    for (int h = lane; h < SG_HASH; h += SG_WAVE) keys[h] = -1;
    if (lane == 0) { count = 0; overflow = 0; npack = 0; }
    __syncthreads();
    sg_insert_row(arp, aci, brp, bci, i, lane, keys, &count, &overflow);
    __syncthreads();
    for (int h = lane; h < SG_HASH; h += SG_WAVE) {
        const int32_t k = keys[h];
        if (k != -1) {
            const int slot = atomicAdd(&npack, 1);
            packed[slot] = k;
        }
    }
    __syncthreads();
    const int m = npack;
    const int64_t base = crp[i];
    // keys are distinct: the rank of a key is its sorted position
    for (int a = lane; a < m; a += SG_WAVE) {
        const int32_t k = packed[a];
        int rank = 0;
        for (int b = 0; b < m; ++b) rank += packed[b] < k;
        cci[base + rank] = k;
    }
}

template <int G>
__global__ void __launch_bounds__(SG_WAVE) sg_numeric_kernel(int64_t n, const int64_t* __restrict__ arp,
                                                             const int32_t* __restrict__ aci,
                                                             const double* __restrict__ aval,
                                                             const int64_t* __restrict__ brp,
                                                             const int32_t* __restrict__ bci,
                                                             const double* __restrict__ bval,
                                                             const int64_t* __restrict__ crp,
                                                             const int32_t* __restrict__ cci,
                                                             double* __restrict__ cval, int cap) {
    extern __shared__ double smem[];
    double* acc = smem;                                      // [G][cap]
    int32_t* cols = reinterpret_cast<int32_t*>(smem + (size_t)G * cap);
    constexpr int GL = SG_WAVE / G;                          // lanes per group
    const int lane = threadIdx.x;
    const int g = lane / GL, gl = lane % GL;
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const int64_t cb = crp[i];
    const int m = (int)(crp[i + 1] - cb);
    for (int a = lane; a < m; a += SG_WAVE) cols[a] = cci[cb + a];
    for (int a = lane; a < G * m; a += SG_WAVE) acc[(a / m) * cap + a % m] = 0.0;
    __syncthreads();
    double* myacc = acc + (size_t)g * cap;
    for (int64_t s = arp[i] + g; s < arp[i + 1]; s += G) {
        const int32_t k = aci[s];
        const double av = aval[s];
        for (int64_t t = brp[k] + gl; t < brp[k + 1]; t += GL) {
            const int32_t j = bci[t];
            int lo = 0, hi = m - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cols[mid] < j) lo = mid + 1; else hi = mid;
            }
            myacc[lo] += av * bval[t];
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    for (int a = lane; a < m; a += SG_WAVE) {
        double v = acc[a];
        for (int gg = 1; gg < G; ++gg) v += acc[(size_t)gg * cap + a];
        cval[cb + a] = v;
    }
}

void spgemm(const DevCSR& A, const DevCSR& B, DevCSR& C, hipStream_t s) {
    GIAMG_REQUIRE(A.ncols == B.nrows, "spgemm: inner dimensions differ");
    const int64_t n = A.nrows;
    C.nrows = n;
    C.ncols = B.ncols;
    C.rp.alloc(n + 1);
    if (n == 0) {
        C.nnz = 0;
        GIAMG_HIP(hipMemsetAsync(C.rp.get(), 0, sizeof(int64_t), s));
        GIAMG_HIP(hipStreamSynchronize(s));
        return;
    }
    DevBuf<int32_t> counts(n);
    GIAMG_REQUIRE(n < (int64_t(1) << 31), "spgemm: too many rows");
    // one wavefront per row: a launch covers at most 2^32 - 1 work-items
    if (n * SG_WAVE > (int64_t)UINT32_MAX)
        throw Error(GIAMG_ENOTSUP, "spgemm: more rows than one launch covers");
    sg_count_kernel<<<(unsigned)n, SG_WAVE, 0, s>>>(n, A.rp.get(), A.ci.get(), B.rp.get(), B.ci.get(),
                                                   counts.get());
    GIAMG_HIP(hipGetLastError());
    std::vector<int32_t> hc(n);
    GIAMG_HIP(hipMemcpyAsync(hc.data(), counts.get(), n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> hrp(n + 1, 0);
    int maxrow = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (hc[r] < 0)
            throw Error(GIAMG_ENOTSUP, "spgemm: a product row has more than " +
                                           std::to_string(SG_MAX_ROW) + " columns");
        hrp[r + 1] = hrp[r] + hc[r];
        maxrow = std::max(maxrow, hc[r]);
    }
    C.nnz = hrp[n];
    GIAMG_REQUIRE(C.nnz < (int64_t(1) << 40), "spgemm: product too large");
    GIAMG_HIP(hipMemcpyAsync(C.rp.get(), hrp.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    C.ci.alloc(C.nnz);
    C.val.alloc(C.nnz);
    if (C.nnz == 0) {
        GIAMG_HIP(hipStreamSynchronize(s));
        setup_row_blocks(C, hrp, s);
        return;
    }
    sg_fill_kernel<<<(unsigned)n, SG_WAVE, 0, s>>>(n, A.rp.get(), A.ci.get(), B.rp.get(), B.ci.get(),
                                                  C.rp.get(), C.ci.get());
    GIAMG_HIP(hipGetLastError());
    const int cap = std::max(1, maxrow);
    if (cap <= 1024) {
        const size_t sm = (size_t)4 * cap * sizeof(double) + (size_t)cap * sizeof(int32_t);
        sg_numeric_kernel<4><<<(unsigned)n, SG_WAVE, sm, s>>>(n, A.rp.get(), A.ci.get(), A.val.get(),
                                                             B.rp.get(), B.ci.get(), B.val.get(),
                                                             C.rp.get(), C.ci.get(), C.val.get(), cap);
    } else {
        const size_t sm = (size_t)cap * sizeof(double) + (size_t)cap * sizeof(int32_t);
        sg_numeric_kernel<1><<<(unsigned)n, SG_WAVE, sm, s>>>(n, A.rp.get(), A.ci.get(), A.val.get(),
                                                             B.rp.get(), B.ci.get(), B.val.get(),
                                                             C.rp.get(), C.ci.get(), C.val.get(), cap);
    }
    GIAMG_HIP(hipGetLastError());
    GIAMG_HIP(hipStreamSynchronize(s));
    setup_row_blocks(C, hrp, s);
}

}  // namespace giamg
