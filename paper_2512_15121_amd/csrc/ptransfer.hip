// p-transfer operators on the device: the rows of P (Algorithms 2-4 and 7:
// each fine node interpolates from the coarse nodes of its elements, a coarse
// node met again in a later element keeps its first weight) and R = P^T.
// The maps (coarse numbering, l2g of the coarse order, the 1-D factor) come
// from the host; the same rows and values as the host build, bit for bit.
//
//  1. counts: one wave per fine row lists the (coarse node, candidate index)
//     pairs of its elements in LDS -- candidate index = element slot of the
//     row x (q+1)^3 + coarse local index, so ascending candidate index is the
//     host's visiting order -- sorts them and counts the distinct nodes;
//  2. fill: the same sort; each distinct node keeps its smallest candidate
//     index, whose weight is I1[i][a] I1[j][b] I1[k][c] in the host's order;
//  3. R: counts per column, a scan, entries placed by atomic counters, then
//     every row of R sorted by column in LDS (so the order of the atomics
//     does not show).
#include "internal.h"
#include "kernels.h"

#include <algorithm>

namespace giamg {

namespace {

constexpr int PT_WAVE = 64;
constexpr int PT_CAND_BITS = 20;   // candidate index bits of a sort key

struct PtArgs {
    int64_t n;                 // fine rows
    int p, q, ncl, p2;         // p2: sort length (power of two >= candidates of any row)
    const uint8_t* free_mask;  // [n]
    const int64_t* nstart;     // [n + 1] node -> element lists
    const int32_t* nel;
    const int32_t* nloc;
    const int32_t* l2g_next;   // [ne][ncl]
    const double* I1;          // [p + 1][q + 1]
    const int64_t* rp;         // fill pass
    int32_t* counts;           // count pass
    int32_t* ci;
    double* val;
    int* err;
};

__device__ void sort_keys(int64_t* keys, int len, int lane) {
    for (int k = 2; k <= len; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < len / 2; t += PT_WAVE) {
                const int i = (t / j) * 2 * j + (t % j);
                const int ixj = i + j;
                const int64_t x = keys[i], y = keys[ixj];
                if ((x > y) == ((i & k) == 0)) {
                    keys[i] = y;
                    keys[ixj] = x;
                }
            }
            __syncthreads();
        }
}

__device__ __forceinline__ int lidx_d(int q, int a, int b, int c) { return ((q + 1) * a + b) * (q + 1) + c; }

// Sorted (coarse node << PT_CAND_BITS | candidate index) keys of row r in
// keys[0 .. len); holes and zero weights are INT64_MAX.  Returns len.
__device__ int row_keys(const PtArgs& a, int64_t r, int64_t* keys, int lane) {
    const int64_t s0 = a.nstart[r], s1 = a.nstart[r + 1];
    const int m = (int)(s1 - s0) * a.ncl;
    int len = PT_WAVE;
    while (len < m) len <<= 1;
    const int q1 = a.q + 1, p1 = a.p + 1;
    for (int t = lane; t < len; t += PT_WAVE) {
        int64_t key = INT64_MAX;
        if (t < m) {
            const int slot = t / a.ncl, cl = t % a.ncl;
            const int64_t e = a.nel[s0 + slot];
            const int loc = a.nloc[s0 + slot];
            const int i = loc / (p1 * p1), j = (loc / p1) % p1, k = loc % p1;
            const int ca = cl / (q1 * q1), cb = (cl / q1) % q1, cc = cl % q1;
            const bool nz = a.I1[i * q1 + ca] != 0.0 && a.I1[j * q1 + cb] != 0.0 && a.I1[k * q1 + cc] != 0.0;
            const int32_t gc = a.l2g_next[e * a.ncl + lidx_d(a.q, ca, cb, cc)];
            if (nz && gc >= 0) key = ((int64_t)gc << PT_CAND_BITS) | t;
        }
        keys[t] = key;
    }
    __syncthreads();
    sort_keys(keys, len, lane);
    return len;
}

__global__ void __launch_bounds__(PT_WAVE) pt_count_kernel(PtArgs a) {
    extern __shared__ int64_t pt_smem[];
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    if (!a.free_mask[r]) {
        if (lane == 0) a.counts[r] = 0;
        return;
    }
    const int len = row_keys(a, r, pt_smem, lane);
    int u = 0;
    for (int c = 0; c < len; c += PT_WAVE) {
        const int i = c + lane;
        const int64_t key = pt_smem[i];
        const bool first = key != INT64_MAX && (i == 0 || (pt_smem[i - 1] >> PT_CAND_BITS) != (key >> PT_CAND_BITS));
        u += __popcll(__ballot(first));
        if (pt_smem[c + PT_WAVE - 1] == INT64_MAX) break;
    }
    if (lane == 0) a.counts[r] = u;
}

__global__ void __launch_bounds__(PT_WAVE) pt_fill_kernel(PtArgs a) {
    extern __shared__ int64_t pt_smem[];
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    if (!a.free_mask[r]) return;
    const int len = row_keys(a, r, pt_smem, lane);
    const int64_t o = a.rp[r], cnt = a.rp[r + 1] - o;
    const int q1 = a.q + 1, p1 = a.p + 1;
    const int64_t s0 = a.nstart[r];
    int u = 0;
    for (int c = 0; c < len; c += PT_WAVE) {
        const int i = c + lane;
        const int64_t key = pt_smem[i];
        const bool first = key != INT64_MAX && (i == 0 || (pt_smem[i - 1] >> PT_CAND_BITS) != (key >> PT_CAND_BITS));
        const uint64_t mask = __ballot(first);
        const int at = u + __popcll(mask & ((1ull << lane) - 1ull));
        if (first && at < cnt) {
            const int t = (int)(key & ((1 << PT_CAND_BITS) - 1));
            const int slot = t / a.ncl, cl = t % a.ncl;
            const int loc = a.nloc[s0 + slot];
            const int ii = loc / (p1 * p1), jj = (loc / p1) % p1, kk = loc % p1;
            const int ca = cl / (q1 * q1), cb = (cl / q1) % q1, cc = cl % q1;
            const double va = a.I1[ii * q1 + ca], vb = a.I1[jj * q1 + cb], vc = a.I1[kk * q1 + cc];
            a.ci[o + at] = (int32_t)(key >> PT_CAND_BITS);
            a.val[o + at] = va * vb * vc;
        }
        u += __popcll(mask);
        if (pt_smem[c + PT_WAVE - 1] == INT64_MAX) break;
    }
    if (lane == 0 && u != cnt) *a.err = 1;
}

// R = P^T: column counts, then entries placed by per-row atomic counters.
__global__ void pt_col_count_kernel(int64_t nnz, const int32_t* __restrict__ ci, int32_t* __restrict__ cnt) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz; t += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(cnt + ci[t], 1);
}

__global__ void pt_scatter_kernel(int64_t n, const int64_t* __restrict__ prp, const int32_t* __restrict__ pci,
                                  const double* __restrict__ pval, const int64_t* __restrict__ rrp,
                                  int32_t* __restrict__ fill, int32_t* __restrict__ rci, double* __restrict__ rval) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        for (int64_t t = prp[r]; t < prp[r + 1]; ++t) {
            const int32_t c = pci[t];
            const int64_t at = rrp[c] + atomicAdd(fill + c, 1);
            rci[at] = (int32_t)r;
            rval[at] = pval[t];
        }
}

// Sort each row of R by column (columns are distinct within a row).
__global__ void __launch_bounds__(PT_WAVE) pt_row_sort_kernel(int64_t nr, const int64_t* __restrict__ rp,
                                                             int32_t* __restrict__ ci, double* __restrict__ val) {
    extern __shared__ int64_t pt_smem[];
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t o = rp[r];
    const int m = (int)(rp[r + 1] - o);
    int len = PT_WAVE;
    while (len < m) len <<= 1;
    int64_t* keys = pt_smem;                                      // column << 32 | position
    double* vals = reinterpret_cast<double*>(pt_smem + len);
    for (int t = lane; t < len; t += PT_WAVE) {
        keys[t] = t < m ? (((int64_t)ci[o + t] << 32) | t) : INT64_MAX;
        if (t < m) vals[t] = val[o + t];
    }
    __syncthreads();
    sort_keys(keys, len, lane);
    for (int t = lane; t < m; t += PT_WAVE) {
        const int64_t k = keys[t];
        ci[o + t] = (int32_t)(k >> 32);
    }
    __syncthreads();
    for (int t = lane; t < m; t += PT_WAVE) val[o + t] = vals[(int)(keys[t] & 0xffffffff)];
}

int pt_lds_limit() {
    int dev = 0, v = 0;
    GIAMG_HIP(hipGetDevice(&dev));
    GIAMG_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    return v;
}

void finish_csr(DevCSR& d, const std::vector<int64_t>& rp, bool make32, hipStream_t s) {
    setup_row_blocks(d, rp, s);
    if (make32) {
        make_fp32_values(d, s);
        setup_row_blocks32(d, rp, s);
    }
}

}  // namespace

void p_transfer_device(const std::vector<int32_t>& l2g, int64_t ne, int p, int q, int64_t n_fine,
                       const std::vector<uint8_t>& free_mask, std::vector<int32_t>& l2g_next,
                       int64_t& n_coarse, int basis, DevCSR& P, DevCSR& R, bool make32, hipStream_t s) {
    const int nl = (p + 1) * (p + 1) * (p + 1), ncl = (q + 1) * (q + 1) * (q + 1);
    GIAMG_REQUIRE((int64_t)l2g.size() == ne * nl, "element map size");
    // node -> element lists of the fine level (entries < 0 belong to no node)
    std::vector<int64_t> nstart(n_fine + 1, 0);
    for (int64_t i = 0; i < ne * nl; ++i)
        if (l2g[i] >= 0) nstart[l2g[i] + 1]++;
    for (int64_t i = 0; i < n_fine; ++i) nstart[i + 1] += nstart[i];
    std::vector<int32_t> nel(nstart.back()), nloc(nstart.back());
    {
        std::vector<int64_t> fill(nstart.begin(), nstart.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int a = 0; a < nl; ++a) {
                const int32_t g = l2g[e * nl + a];
                if (g < 0) continue;
                nel[fill[g]] = (int32_t)e;
                nloc[fill[g]] = a;
                fill[g]++;
            }
    }
    int64_t maxe = 0;
    for (int64_t i = 0; i < n_fine; ++i) maxe = std::max(maxe, nstart[i + 1] - nstart[i]);
    int64_t p2 = PT_WAVE;
    while (p2 < maxe * ncl) p2 <<= 1;
    const int limit = pt_lds_limit();
    if (p2 * 8 > limit || maxe * ncl >= (int64_t(1) << PT_CAND_BITS) || ne >= (int64_t(1) << 31))
        throw Error(GIAMG_ENOTSUP, "device p-transfer: a row's candidates exceed the kernel's LDS list");
    // one wavefront per fine row (and per coarse row in the sort): a launch
    // covers at most 2^32 - 1 work-items
    if (n_fine * PT_WAVE > (int64_t)UINT32_MAX)
        throw Error(GIAMG_ENOTSUP, "device p-transfer: more rows than one launch covers");
    std::vector<double> I1;
    p_transfer_maps(l2g, ne, p, q, n_fine, free_mask, l2g_next, n_coarse, I1, basis);

    DevBuf<uint8_t> dfree(std::max<int64_t>(n_fine, 1));
    DevBuf<int64_t> dnstart(n_fine + 1);
    DevBuf<int32_t> dnel(std::max<size_t>(nel.size(), 1)), dnloc(std::max<size_t>(nloc.size(), 1));
    DevBuf<int32_t> dnext(std::max<size_t>(l2g_next.size(), 1)), counts(std::max<int64_t>(n_fine, 1));
    DevBuf<double> dI1(I1.size());
    DevBuf<int> err(1);
    GIAMG_HIP(hipMemcpyAsync(dfree.get(), free_mask.data(), n_fine, hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dnstart.get(), nstart.data(), (n_fine + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (!nel.empty()) {
        GIAMG_HIP(hipMemcpyAsync(dnel.get(), nel.data(), nel.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        GIAMG_HIP(hipMemcpyAsync(dnloc.get(), nloc.data(), nloc.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    GIAMG_HIP(hipMemcpyAsync(dnext.get(), l2g_next.data(), l2g_next.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dI1.get(), I1.data(), I1.size() * sizeof(double), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemsetAsync(err.get(), 0, sizeof(int), s));

    PtArgs a{};
    a.n = n_fine; a.p = p; a.q = q; a.ncl = ncl; a.p2 = (int)p2;
    a.free_mask = dfree.get(); a.nstart = dnstart.get(); a.nel = dnel.get(); a.nloc = dnloc.get();
    a.l2g_next = dnext.get(); a.I1 = dI1.get(); a.counts = counts.get(); a.err = err.get();
    const size_t lds = (size_t)p2 * 8;
    GIAMG_HIP(hipFuncSetAttribute((const void*)pt_count_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    GIAMG_HIP(hipFuncSetAttribute((const void*)pt_fill_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (n_fine > 0) {
        pt_count_kernel<<<(unsigned)n_fine, PT_WAVE, lds, s>>>(a);
        GIAMG_HIP(hipGetLastError());
    }
    std::vector<int32_t> hc(n_fine);
    if (n_fine > 0)
        GIAMG_HIP(hipMemcpyAsync(hc.data(), counts.get(), n_fine * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> prp(n_fine + 1, 0);
    for (int64_t i = 0; i < n_fine; ++i) prp[i + 1] = prp[i] + hc[i];
    const int64_t nnz = prp[n_fine];

    P.nrows = n_fine;
    P.ncols = n_coarse;
    P.nnz = nnz;
    P.rp.alloc(n_fine + 1);
    P.ci.alloc(std::max<int64_t>(nnz, 1));
    P.val.alloc(std::max<int64_t>(nnz, 1));
    GIAMG_HIP(hipMemcpyAsync(P.rp.get(), prp.data(), (n_fine + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    a.rp = P.rp.get(); a.ci = P.ci.get(); a.val = P.val.get();
    if (n_fine > 0) {
        pt_fill_kernel<<<(unsigned)n_fine, PT_WAVE, lds, s>>>(a);
        GIAMG_HIP(hipGetLastError());
    }

    // R = P^T
    DevBuf<int32_t> ccount(std::max<int64_t>(n_coarse, 1)), cfill(std::max<int64_t>(n_coarse, 1));
    GIAMG_HIP(hipMemsetAsync(ccount.get(), 0, std::max<int64_t>(n_coarse, 1) * sizeof(int32_t), s));
    GIAMG_HIP(hipMemsetAsync(cfill.get(), 0, std::max<int64_t>(n_coarse, 1) * sizeof(int32_t), s));
    if (nnz > 0) {
        pt_col_count_kernel<<<(unsigned)std::min<int64_t>((nnz + 255) / 256, 65536), 256, 0, s>>>(nnz, P.ci.get(),
                                                                                                  ccount.get());
        GIAMG_HIP(hipGetLastError());
    }
    std::vector<int32_t> hcc(std::max<int64_t>(n_coarse, 1));
    int herr = 0;
    GIAMG_HIP(hipMemcpyAsync(hcc.data(), ccount.get(), hcc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipMemcpyAsync(&herr, err.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    if (herr) throw Error(GIAMG_EHIP, "device p-transfer: row counts differ between passes");
    std::vector<int64_t> rrp(n_coarse + 1, 0);
    int64_t rmax = 0;
    for (int64_t i = 0; i < n_coarse; ++i) {
        rrp[i + 1] = rrp[i] + hcc[i];
        rmax = std::max<int64_t>(rmax, hcc[i]);
    }
    int64_t r2 = PT_WAVE;
    while (r2 < rmax) r2 <<= 1;
    if (r2 * 16 > limit) throw Error(GIAMG_ENOTSUP, "device p-transfer: a row of R exceeds the sort's LDS list");
    R.nrows = n_coarse;
    R.ncols = n_fine;
    R.nnz = nnz;
    R.rp.alloc(n_coarse + 1);
    R.ci.alloc(std::max<int64_t>(nnz, 1));
    R.val.alloc(std::max<int64_t>(nnz, 1));
    GIAMG_HIP(hipMemcpyAsync(R.rp.get(), rrp.data(), (n_coarse + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (nnz > 0) {
        pt_scatter_kernel<<<(unsigned)std::min<int64_t>((n_fine + 255) / 256, 65536), 256, 0, s>>>(
            n_fine, P.rp.get(), P.ci.get(), P.val.get(), R.rp.get(), cfill.get(), R.ci.get(), R.val.get());
        GIAMG_HIP(hipGetLastError());
        const size_t slds = (size_t)r2 * 16;
        GIAMG_HIP(hipFuncSetAttribute((const void*)pt_row_sort_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)slds));
        pt_row_sort_kernel<<<(unsigned)n_coarse, PT_WAVE, slds, s>>>(n_coarse, R.rp.get(), R.ci.get(), R.val.get());
        GIAMG_HIP(hipGetLastError());
    }
    GIAMG_HIP(hipStreamSynchronize(s));
    finish_csr(P, prp, make32, s);
    finish_csr(R, rrp, make32, s);
}

}  // namespace giamg
