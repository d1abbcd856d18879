// Fine-level assembly on the device: A = K + lambda M for Q_p hexahedra under
// the trilinear map of their corners, integrated with p + 2 Gauss points per
// direction (the Helmholtz problem of Section 3.1), in CSR over all nodes:
// a free row holds every free node of the elements around it, a constrained
// row is the identity.  Same pattern and entry order as the host assembly;
// each entry is summed over its elements in ascending element order.
//
// Three kernels:
//  1. geometry: per element and quadrature point the six entries of
//     w |J| J^-1 J^-T and the mass weight lambda w |J|;
//  2. counts: one wave per row sorts the row's candidate columns (the nodes
//     of its elements) in LDS and counts the distinct free ones;
//  3. fill: the same sort gives the row's columns; then, element by element
//     in ascending order, the row of the element matrix belonging to the
//     row's local node is formed by sum factorisation (the local node's
//     gradient weighted by the geometric factors at the quadrature points,
//     contracted with the 1-D tables one direction at a time: z, then y,
//     then x) and added into the row's LDS accumulators.
#include "internal.h"
#include "kernels.h"

#include <algorithm>

namespace giamg {

namespace {

constexpr int ASM_WAVE = 64;   // one wave per row
constexpr int GEOM_THREADS = 256;

struct AsmArgs {
    int64_t n, ne;
    int n1, nq, nl, Q;
    int p2;                           // sort length (power of two >= candidates of any row)
    int umax;                         // most columns of a row (fill pass)
    const int32_t* l2g;               // [ne][nl]
    const uint8_t* cons;              // [n]
    const int64_t* nstart;            // [n + 1]
    const int32_t* nel;               // elements of each node, ascending
    const int32_t* nloc;              // local index of the node in each of them
    const double* tabs;               // L[n1][nq] then D[n1][nq]
    const double* G;                  // [ne][Q][7]
    const int64_t* rp;                // fill pass
    int32_t* counts;                  // count pass
    int32_t* ci;
    double* val;
    int* err;                         // [0]: a row's count changed between the passes
};

// Bitonic sort of keys[0 .. len) (len a power of two) by one wave.
__device__ void wave_sort(int32_t* keys, int len, int lane) {
    for (int k = 2; k <= len; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < len / 2; t += ASM_WAVE) {
                const int i = (t / j) * 2 * j + (t % j);
                const int ixj = i + j;
                const int32_t x = keys[i], y = keys[ixj];
                const bool up = (i & k) == 0;
                if ((x > y) == up) {
                    keys[i] = y;
                    keys[ixj] = x;
                }
            }
            __syncthreads();
        }
}

// The row's candidate columns (every node of every element of the row,
// constrained nodes as INT32_MAX) sorted into keys[0 .. len); returns len.
__device__ int row_candidates(const AsmArgs& a, int64_t r, int32_t* keys, int lane) {
    const int64_t s0 = a.nstart[r], s1 = a.nstart[r + 1];
    const int m = (int)(s1 - s0) * a.nl;
    int len = ASM_WAVE;
    while (len < m) len <<= 1;
    for (int t = lane; t < len; t += ASM_WAVE) {
        int32_t key = INT32_MAX;
        if (t < m) {
            const int64_t s = s0 + t / a.nl;
            const int32_t g = a.l2g[(int64_t)a.nel[s] * a.nl + t % a.nl];
            key = a.cons[g] ? INT32_MAX : g;
        }
        keys[t] = key;
    }
    __syncthreads();
    wave_sort(keys, len, lane);
    return len;
}

// Distinct keys below INT32_MAX of the sorted keys[0 .. len), the first cap
// of them written to cols (if not null) in ascending order; returns their
// number.
__device__ int distinct_keys(const int32_t* keys, int len, int32_t* cols, int cap, int lane) {
    int u = 0;
    for (int c = 0; c < len; c += ASM_WAVE) {
        const int i = c + lane;
        const int32_t key = keys[i];
        const bool first = key != INT32_MAX && (i == 0 || keys[i - 1] != key);
        const uint64_t mask = __ballot(first);
        const int at = u + __popcll(mask & ((1ull << lane) - 1ull));
        if (first && cols && at < cap) cols[at] = key;
        u += __popcll(mask);
        if (keys[c + ASM_WAVE - 1] == INT32_MAX) break;   // sorted: the rest are constrained or padding
    }
    return u;
}

__global__ void __launch_bounds__(GEOM_THREADS) asm_geometry_kernel(int64_t ne, int nq, const double* __restrict__ corners,
                                                                    const double* __restrict__ gq,
                                                                    const double* __restrict__ wq, double lambda,
                                                                    double* __restrict__ G, int* __restrict__ bad) {
    const int Q = nq * nq * nq;
    const int64_t t = (int64_t)blockIdx.x * GEOM_THREADS + threadIdx.x;
    if (t >= ne * Q) return;
    const int64_t e = t / Q;
    const int q = (int)(t % Q);
    const int qx = q / (nq * nq), qy = (q / nq) % nq, qz = q % nq;
    const double xi[3] = {gq[qx], gq[qy], gq[qz]};
    const double* X = corners + e * 24;
    // Jacobian of the trilinear map: J[a][d] = d x_a / d xi_d
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int c = 0; c < 8; ++c) {
        const double sx = ((c >> 2) & 1) ? 1.0 : -1.0, sy = ((c >> 1) & 1) ? 1.0 : -1.0,
                     sz = (c & 1) ? 1.0 : -1.0;
        const double fx = 0.5 * (1 + sx * xi[0]), fy = 0.5 * (1 + sy * xi[1]), fz = 0.5 * (1 + sz * xi[2]);
        const double dN[3] = {0.5 * sx * fy * fz, 0.5 * sy * fx * fz, 0.5 * sz * fx * fy};
        for (int r = 0; r < 3; ++r)
            for (int d = 0; d < 3; ++d) J[r][d] += X[c * 3 + r] * dN[d];
    }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0.0)) {
        *bad = 1;
        return;
    }
    // inverse: Ji[d][r] = d xi_d / d x_r
    double Ji[3][3];
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    const double w = wq[qx] * wq[qy] * wq[qz] * det;
    double* g = G + t * 7;
    int m = 0;
    for (int d = 0; d < 3; ++d)
        for (int f = d; f < 3; ++f) {
            double s = 0.0;
            for (int r = 0; r < 3; ++r) s += Ji[d][r] * Ji[f][r];
            g[m++] = w * s;      // xx, xy, xz, yy, yz, zz
        }
    g[6] = lambda * w;
}

__global__ void __launch_bounds__(ASM_WAVE) asm_count_kernel(AsmArgs a) {
    extern __shared__ double smem[];
    int32_t* keys = reinterpret_cast<int32_t*>(smem);
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    if (a.cons[r]) {
        if (lane == 0) a.counts[r] = 1;
        return;
    }
    const int len = row_candidates(a, r, keys, lane);
    const int u = distinct_keys(keys, len, nullptr, 0, lane);
    if (lane == 0) a.counts[r] = u;
}

// Row `a_loc` of the element matrix of element e into kr[0 .. nl) (LDS),
// with work (LDS) of 4 Q + 3 nq^2 n1 doubles.  Ends with a barrier.
__device__ void element_row(const AsmArgs& a, int64_t e, int a_loc, const double* TL, const double* TD,
                            double* work, double* kr_out, int lane) {
    const int n1 = a.n1, nq = a.nq, Q = a.Q;
    const int i = a_loc / (n1 * n1), j = (a_loc / n1) % n1, k = a_loc % n1;
    double* Hx = work;
    double* Hy = Hx + Q;
    double* Hz = Hy + Q;
    double* Hm = Hz + Q;
    double* U = Hm + Q;                       // [3][nq][nq][n1]
    const int usz = nq * nq * n1;
    // A: gradient of the local function weighted by the geometric factors
    const double* Ge = a.G + e * (int64_t)Q * 7;
    for (int q = lane; q < Q; q += ASM_WAVE) {
        const int qx = q / (nq * nq), qy = (q / nq) % nq, qz = q % nq;
        const double Li = TL[i * nq + qx], Di = TD[i * nq + qx];
        const double Lj = TL[j * nq + qy], Dj = TD[j * nq + qy];
        const double Lk = TL[k * nq + qz], Dk = TD[k * nq + qz];
        const double gx = Di * Lj * Lk, gy = Li * Dj * Lk, gz = Li * Lj * Dk;
        const double* g = Ge + (int64_t)q * 7;
        Hx[q] = g[0] * gx + g[1] * gy + g[2] * gz;
        Hy[q] = g[1] * gx + g[3] * gy + g[4] * gz;
        Hz[q] = g[2] * gx + g[4] * gy + g[5] * gz;
        Hm[q] = g[6] * (Li * Lj * Lk);
    }
    __syncthreads();
    // B: contract z -- x and y fields with L, the z field with D plus the mass field with L
    for (int t = lane; t < 3 * usz; t += ASM_WAVE) {
        const int f = t / usz, rem = t % usz, qxy = rem / n1, kp = rem % n1;
        const double* l = TL + kp * nq;
        double s = 0.0;
        if (f == 0) {
            for (int qz = 0; qz < nq; ++qz) s += l[qz] * Hx[qxy * nq + qz];
        } else if (f == 1) {
            for (int qz = 0; qz < nq; ++qz) s += l[qz] * Hy[qxy * nq + qz];
        } else {
            const double* dd = TD + kp * nq;
            for (int qz = 0; qz < nq; ++qz) s += dd[qz] * Hz[qxy * nq + qz] + l[qz] * Hm[qxy * nq + qz];
        }
        U[f * usz + qxy * n1 + kp] = s;
    }
    __syncthreads();
    // C: contract y -- the x field with L; the y field with D plus the z and mass fields with L
    double* V = work;                          // [2][nq][n1][n1] over the dead H fields
    const int vsz = nq * n1 * n1;
    for (int t = lane; t < 2 * vsz; t += ASM_WAVE) {
        const int f = t / vsz, rem = t % vsz, qx = rem / (n1 * n1), jp = (rem / n1) % n1, kp = rem % n1;
        const double* l = TL + jp * nq;
        double s = 0.0;
        if (f == 0) {
            for (int qy = 0; qy < nq; ++qy) s += l[qy] * U[(qx * nq + qy) * n1 + kp];
        } else {
            const double* dd = TD + jp * nq;
            for (int qy = 0; qy < nq; ++qy)
                s += dd[qy] * U[usz + (qx * nq + qy) * n1 + kp] + l[qy] * U[2 * usz + (qx * nq + qy) * n1 + kp];
        }
        V[f * vsz + (qx * n1 + jp) * n1 + kp] = s;
    }
    __syncthreads();
    // D: contract x -- the x field with D, the rest with L
    for (int b = lane; b < a.nl; b += ASM_WAVE) {
        const int ip = b / (n1 * n1), jk = b % (n1 * n1);
        const double* l = TL + ip * nq;
        const double* dd = TD + ip * nq;
        double s = 0.0;
        for (int qx = 0; qx < nq; ++qx) s += dd[qx] * V[qx * n1 * n1 + jk] + l[qx] * V[vsz + qx * n1 * n1 + jk];
        kr_out[b] = s;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(ASM_WAVE) asm_fill_kernel(AsmArgs a) {
    extern __shared__ double smem[];
    const int tsz = a.n1 * a.nq;
    double* vals = smem;                                   // [umax]
    double* TL = vals + a.umax;                            // [n1][nq]
    double* TD = TL + tsz;
    double* work = TD + tsz;                               // max(p2 ints, 4 Q + 3 nq^2 n1 doubles)
    const int wsz = max((a.p2 + 1) / 2, 4 * a.Q + 3 * a.nq * a.nq * a.n1);
    double* kr = work + 4 * a.Q;                           // element row over the U area after step C
    int32_t* cols = reinterpret_cast<int32_t*>(work + wsz);   // [umax]
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t o = a.rp[r];
    if (a.cons[r]) {
        if (lane == 0) {
            a.ci[o] = (int32_t)r;
            a.val[o] = 1.0;
        }
        return;
    }
    for (int t = lane; t < 2 * tsz; t += ASM_WAVE) TL[t] = a.tabs[t];
    const int len = row_candidates(a, r, reinterpret_cast<int32_t*>(work), lane);
    const int u = distinct_keys(reinterpret_cast<const int32_t*>(work), len, cols, a.umax, lane);
    if (u != (int)(a.rp[r + 1] - o)) {
        if (lane == 0) *a.err = 1;
        return;
    }
    for (int t = lane; t < u; t += ASM_WAVE) {
        a.ci[o + t] = cols[t];
        vals[t] = 0.0;
    }
    __syncthreads();
    for (int64_t s = a.nstart[r]; s < a.nstart[r + 1]; ++s) {
        const int64_t e = a.nel[s];
        element_row(a, e, a.nloc[s], TL, TD, work, kr, lane);
        const int32_t* g = a.l2g + e * a.nl;
        for (int b = lane; b < a.nl; b += ASM_WAVE) {
            const int32_t c = g[b];
            if (a.cons[c]) continue;
            int lo = 0, hi = u - 1;           // c is among the row's columns
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cols[mid] < c) lo = mid + 1;
                else hi = mid;
            }
            vals[lo] += kr[b];
        }
        __syncthreads();
    }
    for (int t = lane; t < u; t += ASM_WAVE) a.val[o + t] = vals[t];
}

int lds_limit() {
    int dev = 0, v = 0;
    GIAMG_HIP(hipGetDevice(&dev));
    GIAMG_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    return v;
}

}  // namespace

void assemble_fine_device(const std::vector<double>& corners, const int32_t* l2g, int64_t ne, int p,
                          int64_t n, double lambda, const std::vector<uint8_t>& cons, int basis, DevCSR& d,
                          hipStream_t s) {
    const int n1 = p + 1, nq = p + 2, nl = n1 * n1 * n1, Q = nq * nq * nq;
    GIAMG_REQUIRE(n < (int64_t(1) << 31), "too many nodes for 32-bit column ids");
    // one wavefront per row: a launch covers at most 2^32 - 1 work-items
    if (n * ASM_WAVE > (int64_t)UINT32_MAX)
        throw Error(GIAMG_ENOTSUP, "device assembly: more rows than one launch covers");
    std::vector<int64_t> nstart;
    std::vector<int32_t> nel, nloc;
    node_elements(l2g, ne, nl, n, nstart, nel, nloc);
    int64_t maxe = 0;
    for (int64_t i = 0; i < n; ++i) {
        maxe = std::max(maxe, nstart[i + 1] - nstart[i]);
        // a node listed twice by one element: the element-row scatter adds a
        // row's entries of one element in parallel, so they must be distinct
        for (int64_t s = nstart[i] + 1; s < nstart[i + 1]; ++s)
            if (nel[s] == nel[s - 1])
                throw Error(GIAMG_ENOTSUP, "device assembly: an element lists a node twice");
    }
    int64_t p2 = ASM_WAVE;
    while (p2 < maxe * nl) p2 <<= 1;
    const int limit = lds_limit();
    const int64_t work_doubles = std::max<int64_t>((p2 + 1) / 2, 4 * (int64_t)Q + 3 * (int64_t)nq * nq * n1);
    if (p2 * 4 > limit || work_doubles * 8 + 2 * (int64_t)n1 * nq * 8 > limit)
        throw Error(GIAMG_ENOTSUP, "device assembly: a row's elements exceed the kernels' LDS lists");

    std::vector<double> L, D, gq, wq;
    reference_tables(p, basis, L, D, gq, wq);
    std::vector<double> tabs(L);
    tabs.insert(tabs.end(), D.begin(), D.end());

    DevBuf<int32_t> dl2g(ne * nl);
    DevBuf<double> dcorn(ne * 24), dtabs(tabs.size()), dg(nq), dw(nq), G(ne * (int64_t)Q * 7);
    DevBuf<uint8_t> dcons(n);
    DevBuf<int64_t> dnstart(n + 1);
    DevBuf<int32_t> dnel(nel.size()), dnloc(nloc.size()), counts(n);
    DevBuf<int> flags(2);
    GIAMG_HIP(hipMemcpyAsync(dl2g.get(), l2g, ne * nl * sizeof(int32_t), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dcorn.get(), corners.data(), ne * 24 * sizeof(double), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dtabs.get(), tabs.data(), tabs.size() * sizeof(double), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dg.get(), gq.data(), nq * sizeof(double), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dw.get(), wq.data(), nq * sizeof(double), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dcons.get(), cons.data(), n, hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dnstart.get(), nstart.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dnel.get(), nel.data(), nel.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dnloc.get(), nloc.data(), nloc.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemsetAsync(flags.get(), 0, 2 * sizeof(int), s));

    const int64_t gthreads = ne * (int64_t)Q;
    asm_geometry_kernel<<<(unsigned)((gthreads + GEOM_THREADS - 1) / GEOM_THREADS), GEOM_THREADS, 0, s>>>(
        ne, nq, dcorn.get(), dg.get(), dw.get(), lambda, G.get(), flags.get());
    GIAMG_HIP(hipGetLastError());

    AsmArgs a{};
    a.n = n; a.ne = ne; a.n1 = n1; a.nq = nq; a.nl = nl; a.Q = Q; a.p2 = (int)p2;
    a.l2g = dl2g.get(); a.cons = dcons.get(); a.nstart = dnstart.get(); a.nel = dnel.get();
    a.nloc = dnloc.get(); a.tabs = dtabs.get(); a.G = G.get(); a.counts = counts.get();
    a.err = flags.get() + 1;
    const size_t count_lds = (size_t)p2 * 4;
    GIAMG_HIP(hipFuncSetAttribute((const void*)asm_count_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)count_lds));
    asm_count_kernel<<<(unsigned)n, ASM_WAVE, count_lds, s>>>(a);
    GIAMG_HIP(hipGetLastError());
    std::vector<int32_t> hc(n);
    int hflags[2] = {0, 0};
    GIAMG_HIP(hipMemcpyAsync(hc.data(), counts.get(), n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipMemcpyAsync(hflags, flags.get(), 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    if (hflags[0]) throw Error(GIAMG_EINVAL, "non-positive Jacobian determinant in an element");
    std::vector<int64_t> rp(n + 1, 0);
    int umax = 1;
    for (int64_t i = 0; i < n; ++i) {
        rp[i + 1] = rp[i] + hc[i];
        umax = std::max(umax, hc[i]);
    }
    const int64_t fill_lds = (int64_t)umax * 8 + 2 * (int64_t)n1 * nq * 8 + work_doubles * 8 + (int64_t)umax * 4;
    if (fill_lds > limit)
        throw Error(GIAMG_ENOTSUP, "device assembly: a row's columns exceed the kernels' LDS lists");

    d.nrows = d.ncols = n;
    d.nnz = rp[n];
    d.rp.alloc(n + 1);
    d.ci.alloc(std::max<int64_t>(d.nnz, 1));
    d.val.alloc(std::max<int64_t>(d.nnz, 1));
    GIAMG_HIP(hipMemcpyAsync(d.rp.get(), rp.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    a.umax = umax;
    a.rp = d.rp.get(); a.ci = d.ci.get(); a.val = d.val.get();
    GIAMG_HIP(hipFuncSetAttribute((const void*)asm_fill_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)fill_lds));
    asm_fill_kernel<<<(unsigned)n, ASM_WAVE, (size_t)fill_lds, s>>>(a);
    GIAMG_HIP(hipGetLastError());
    GIAMG_HIP(hipMemcpyAsync(hflags, flags.get(), 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    GIAMG_HIP(hipStreamSynchronize(s));
    if (hflags[1]) throw Error(GIAMG_EHIP, "device assembly: row counts differ between passes");
    setup_row_blocks(d, rp, s);
}

}  // namespace giamg
