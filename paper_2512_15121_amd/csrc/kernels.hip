// Device kernels of the GIAMG solve phase for gfx950 (CDNA4).
//
// The solve is HBM-bound sparse work: CSR products of the level operators
// (Algorithm 1: smoothing, residual, restriction, prolongation), vector
// updates and dot products of CG.  Design:
//  * one 64-lane wavefront per row, rows of a block contiguous, CSR values
//    and column indices streamed with non-temporal loads so the cache keeps
//    the gathered vector;
//  * blocks remapped so each of the eight XCDs works on a contiguous slice
//    of rows (its L2 then holds the slice of the gathered vector);
//  * every smoother/CG vector update fused into the product's row epilogue;
//  * reductions are two-stage and fixed-order (no floating-point atomics), so
//    results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace giamg {

constexpr int WAVE = 64;
constexpr int SPMV_WAVES = 4;                   // waves per block
constexpr int SPMV_RPW = 4;                     // consecutive rows per wave
constexpr int SPMV_ROWS = SPMV_WAVES * SPMV_RPW;
constexpr int VEC_THREADS = 256;
constexpr int64_t VEC_MAX_BLOCKS = 2048;
constexpr int RED_THREADS = 1024;

// Hardware dispatches block b to XCD (b mod 8).  Logical block ids are
// reassigned so that each XCD receives one contiguous range.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
    int64_t x = b & 7, i = b >> 3, q = G >> 3, r = G & 7;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

template <typename T>
__device__ __forceinline__ T ldnt(const T* p) {
    return __builtin_nontemporal_load(p);
}

int64_t spmv_blocks(int64_t n) { return (n + SPMV_ROWS - 1) / SPMV_ROWS; }

// Row-sum of the CSR product for one row, all lanes receive the result.
template <typename T>
__device__ __forceinline__ T row_dot(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                     const T* __restrict__ val, const T* __restrict__ v,
                                     int64_t row, int lane) {
    const int64_t s = rp[row], e = rp[row + 1];
    T acc0 = 0, acc1 = 0;
    int64_t j = s + lane;
    for (; j + WAVE < e; j += 2 * WAVE) {
        const int32_t c0 = ldnt(ci + j), c1 = ldnt(ci + j + WAVE);
        const T a0 = ldnt(val + j), a1 = ldnt(val + j + WAVE);
        acc0 += a0 * v[c0];
        acc1 += a1 * v[c1];
    }
    if (j < e) acc0 += ldnt(val + j) * v[ldnt(ci + j)];
    return wave_sum(acc0 + acc1);
}

template <typename T, int MODE>
__global__ void __launch_bounds__(SPMV_WAVES* WAVE) spmv_kernel(SpmvArgs<T> a) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row0 = (lb * SPMV_WAVES + wave) * SPMV_RPW;
    double dot = 0.0;
    for (int k = 0; k < SPMV_RPW; ++k) {
        const int64_t row = row0 + k;
        if (row >= a.n) break;
        const T y = row_dot(a.rp, a.ci, a.val, a.v, row, lane);
        if (lane == 0) {
            if constexpr (MODE == SPMV_PLAIN) {
                a.y[row] = y;
            } else if constexpr (MODE == SPMV_RESID) {
                a.y[row] = a.f[row] - y;
            } else if constexpr (MODE == SPMV_ADD) {
                a.y[row] += y;
            } else if constexpr (MODE == SPMV_CHEB_INIT) {
                const T res = a.dinv[row] * (a.f[row] - y);
                a.r[row] = res;
                a.y[row] = res * a.inv_theta;
            } else if constexpr (MODE == SPMV_CHEB_STEP) {
                const T rr = a.r[row] - a.dinv[row] * y;
                const T dold = a.v[row];
                const T dn = a.c1 * dold + a.c2 * rr;
                a.r[row] = rr;
                a.y[row] = dn;
                const T inc = (a.flags & CHEB_LAST) ? dold + dn : dold;
                if (a.flags & CHEB_ASSIGN)
                    a.x[row] = inc;
                else
                    a.x[row] += inc;
            } else if constexpr (MODE == SPMV_JACOBI) {
                a.y[row] = a.v[row] + a.omega * a.dinv[row] * (a.f[row] - y);
            } else if constexpr (MODE == SPMV_DOT) {
                a.y[row] = y;
                dot += (double)a.v[row] * (double)y;
            } else if constexpr (MODE == SPMV_DINV) {
                a.y[row] = a.dinv[row] * y;
            }
        }
    }
    if constexpr (MODE == SPMV_DOT) {
        __shared__ double red[SPMV_WAVES];
        if (lane == 0) red[wave] = dot;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < SPMV_WAVES; ++w) s += red[w];
            a.partial[lb] = s;
        }
    }
}

template <typename T>
void launch_spmv(int mode, const SpmvArgs<T>& a, hipStream_t s) {
    if (a.n <= 0) return;
    const dim3 grid((unsigned)spmv_blocks(a.n)), block(SPMV_WAVES * WAVE);
    switch (mode) {
        case SPMV_PLAIN: spmv_kernel<T, SPMV_PLAIN><<<grid, block, 0, s>>>(a); break;
        case SPMV_RESID: spmv_kernel<T, SPMV_RESID><<<grid, block, 0, s>>>(a); break;
        case SPMV_ADD: spmv_kernel<T, SPMV_ADD><<<grid, block, 0, s>>>(a); break;
        case SPMV_CHEB_INIT: spmv_kernel<T, SPMV_CHEB_INIT><<<grid, block, 0, s>>>(a); break;
        case SPMV_CHEB_STEP: spmv_kernel<T, SPMV_CHEB_STEP><<<grid, block, 0, s>>>(a); break;
        case SPMV_JACOBI: spmv_kernel<T, SPMV_JACOBI><<<grid, block, 0, s>>>(a); break;
        case SPMV_DOT: spmv_kernel<T, SPMV_DOT><<<grid, block, 0, s>>>(a); break;
        case SPMV_DINV: spmv_kernel<T, SPMV_DINV><<<grid, block, 0, s>>>(a); break;
        default: throw Error(GIAMG_EINVAL, "unknown product mode");
    }
    GIAMG_HIP(hipGetLastError());
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
                                  T inv_theta, int write_x) {
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
    cheb_init0_kernel<T><<<vgrid(n), VEC_THREADS, 0, s>>>(n, f, dinv, r, d, x, inv_theta, write_x);
    GIAMG_HIP(hipGetLastError());
}
template void launch_cheb_init0<double>(int64_t, const double*, const double*, double*, double*,
                                        double*, double, bool, hipStream_t);
template void launch_cheb_init0<float>(int64_t, const float*, const float*, float*, float*, float*,
                                       float, bool, hipStream_t);

template <typename T>
__global__ void jacobi0_kernel(int64_t n, const T* __restrict__ f, const T* __restrict__ dinv,
                               T* __restrict__ x, T omega) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = omega * dinv[i] * f[i];
}
template <typename T>
void launch_jacobi0(int64_t n, const T* f, const T* dinv, T* x, T omega, hipStream_t s) {
    if (n <= 0) return;
    jacobi0_kernel<T><<<vgrid(n), VEC_THREADS, 0, s>>>(n, f, dinv, x, omega);
    GIAMG_HIP(hipGetLastError());
}
template void launch_jacobi0<double>(int64_t, const double*, const double*, double*, double,
                                     hipStream_t);
template void launch_jacobi0<float>(int64_t, const float*, const float*, float*, float, hipStream_t);

template <typename T>
__global__ void copy_kernel(int64_t n, const T* __restrict__ a, T* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}
template <typename T>
void launch_copy(int64_t n, const T* a, T* b, hipStream_t s) {
    if (n <= 0) return;
    copy_kernel<T><<<vgrid(n), VEC_THREADS, 0, s>>>(n, a, b);
    GIAMG_HIP(hipGetLastError());
}
template void launch_copy<double>(int64_t, const double*, double*, hipStream_t);
template void launch_copy<float>(int64_t, const float*, float*, hipStream_t);

template <typename T>
__global__ void add_kernel(int64_t n, const T* __restrict__ a, T* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] += a[i];
}
template <typename T>
void launch_add(int64_t n, const T* a, T* b, hipStream_t s) {
    if (n <= 0) return;
    add_kernel<T><<<vgrid(n), VEC_THREADS, 0, s>>>(n, a, b);
    GIAMG_HIP(hipGetLastError());
}
template void launch_add<double>(int64_t, const double*, double*, hipStream_t);
template void launch_add<float>(int64_t, const float*, float*, hipStream_t);

template <typename Tin, typename Tout>
__global__ void convert_kernel(int64_t n, const Tin* __restrict__ a, Tout* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (Tout)a[i];
}
template <typename Tin, typename Tout>
void launch_convert(int64_t n, const Tin* a, Tout* b, hipStream_t s) {
    if (n <= 0) return;
    convert_kernel<Tin, Tout><<<vgrid(n), VEC_THREADS, 0, s>>>(n, a, b);
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
                                                     const T* __restrict__ f, T* __restrict__ x) {
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
    coarse_kernel<T><<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, inv, f, x);
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

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int o = NT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(VEC_THREADS) dot_partial_kernel(int64_t n, const double* __restrict__ a,
                                                                  const double* __restrict__ b,
                                                                  double* __restrict__ partial) {
    __shared__ double sh[VEC_THREADS];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VEC_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VEC_THREADS)
        s += a[i] * b[i];
    s = block_sum<VEC_THREADS>(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
void launch_dot_partial(int64_t n, const double* a, const double* b, double* partial,
                        hipStream_t s) {
    dot_partial_kernel<<<(unsigned)vec_blocks(n), VEC_THREADS, 0, s>>>(n, a, b, partial);
    GIAMG_HIP(hipGetLastError());
}

__global__ void __launch_bounds__(VEC_THREADS) dot2_partial_kernel(int64_t n, const double* __restrict__ a,
                                                                   const double* __restrict__ b,
                                                                   const double* __restrict__ c,
                                                                   double* __restrict__ partial) {
    __shared__ double sh[VEC_THREADS];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VEC_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VEC_THREADS) {
        s0 += a[i] * b[i];
        s1 += c[i] * b[i];
    }
    s0 = block_sum<VEC_THREADS>(s0, sh);
    s1 = block_sum<VEC_THREADS>(s1, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s0;
        partial[gridDim.x + blockIdx.x] = s1;
    }
}
void launch_dot2_partial(int64_t n, const double* a, const double* b, const double* c,
                         double* partial, hipStream_t s) {
    dot2_partial_kernel<<<(unsigned)vec_blocks(n), VEC_THREADS, 0, s>>>(n, a, b, c, partial);
    GIAMG_HIP(hipGetLastError());
}

// out[c] = sum_{i<m} partial[c*stride + i] for c < ncomp, fixed order.
__global__ void __launch_bounds__(RED_THREADS) reduce_kernel(int64_t m, const double* __restrict__ partial,
                                                             int64_t stride, int ncomp,
                                                             double* __restrict__ out) {
    __shared__ double sh[RED_THREADS];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int64_t i = threadIdx.x; i < m; i += RED_THREADS) s += partial[c * stride + i];
        s = block_sum<RED_THREADS>(s, sh);
        if (threadIdx.x == 0) out[c] = s;
    }
}
void launch_reduce(int64_t m, const double* partial, int64_t stride, int ncomp, double* out,
                   hipStream_t s) {
    reduce_kernel<<<1, RED_THREADS, 0, s>>>(m, partial, stride, ncomp, out);
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
                                                                 double* __restrict__ partial) {
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
    pcg_update_kernel<<<(unsigned)vec_blocks(n), VEC_THREADS, 0, s>>>(n, x, r, rold, p, q, scal, partial);
    GIAMG_HIP(hipGetLastError());
}

__global__ void pcg_direction_kernel(int64_t n, const double* __restrict__ z, double* __restrict__ p,
                                     const double* __restrict__ scal) {
    const double beta = scal[S_BETA];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
}
void launch_pcg_direction(int64_t n, const double* z, double* p, const double* scal, hipStream_t s) {
    pcg_direction_kernel<<<vgrid(n), VEC_THREADS, 0, s>>>(n, z, p, scal);
    GIAMG_HIP(hipGetLastError());
}

__global__ void pcg_alpha_kernel(double* scal) {
    const double pq = scal[S_PQ];
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(scal[S_RZ])) {
        scal[S_FLAG] = 1.0;
        scal[S_ALPHA] = 0.0;
    } else {
        scal[S_ALPHA] = scal[S_RZ] / pq;
    }
}
void launch_pcg_alpha(double* scal, hipStream_t s) {
    pcg_alpha_kernel<<<1, 1, 0, s>>>(scal);
    GIAMG_HIP(hipGetLastError());
}

__global__ void pcg_beta_kernel(double* scal, int flexible, int first) {
    const double rzn = scal[S_RZNEW];
    if (first) {
        scal[S_BETA] = 0.0;
    } else if (flexible) {
        scal[S_BETA] = (rzn - scal[S_ZROLD]) / scal[S_RZ];
    } else {
        scal[S_BETA] = rzn / scal[S_RZ];
    }
    if (!isfinite(rzn)) scal[S_FLAG] = 1.0;
    scal[S_RZ] = rzn;
}
void launch_pcg_beta(double* scal, bool flexible, bool first, hipStream_t s) {
    pcg_beta_kernel<<<1, 1, 0, s>>>(scal, flexible ? 1 : 0, first ? 1 : 0);
    GIAMG_HIP(hipGetLastError());
}

// r = b - A x with block partials of b.b (first half) and r.r (second half)
__global__ void __launch_bounds__(SPMV_WAVES* WAVE) residual_init_kernel(
    int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const double* __restrict__ val, const double* __restrict__ b, const double* __restrict__ x,
    double* __restrict__ r, double* __restrict__ partial) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row0 = (lb * SPMV_WAVES + wave) * SPMV_RPW;
    double bb = 0.0, rr = 0.0;
    for (int k = 0; k < SPMV_RPW; ++k) {
        const int64_t row = row0 + k;
        if (row >= n) break;
        const double y = row_dot(rp, ci, val, x, row, lane);
        if (lane == 0) {
            const double bi = b[row];
            const double ri = bi - y;
            r[row] = ri;
            bb += bi * bi;
            rr += ri * ri;
        }
    }
    __shared__ double red[2][SPMV_WAVES];
    if (lane == 0) {
        red[0][wave] = bb;
        red[1][wave] = rr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < SPMV_WAVES; ++w) {
            s0 += red[0][w];
            s1 += red[1][w];
        }
        partial[lb] = s0;
        partial[gridDim.x + lb] = s1;
    }
}
void launch_residual_init(int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                          const double* b, const double* x, double* r, double* partial,
                          hipStream_t s) {
    residual_init_kernel<<<(unsigned)spmv_blocks(n), SPMV_WAVES * WAVE, 0, s>>>(n, rp, ci, val, b, x,
                                                                                r, partial);
    GIAMG_HIP(hipGetLastError());
}

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
