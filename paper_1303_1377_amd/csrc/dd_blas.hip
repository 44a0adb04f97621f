// dd_blas.hip -- vector algebra for the Krylov solvers (FGMRES / GMRES).
//
// The Arnoldi step needs the inner products V_i^H w of one new vector against
// all basis vectors, then w -= V h and ||w||.  Both are single kernels: every
// thread keeps one accumulator per basis vector while streaming w once, the
// workgroup partials are written to a work buffer, and the last workgroup to
// finish (atomic ticket) adds the partials in a fixed order, so results do not
// depend on scheduling.  Accumulation is FP64 for every storage precision.
#include "dd_kernels.h"

namespace dd {

static constexpr int MAXM = 32;      // basis vectors handled per call
static constexpr int RED_WG = 512;   // workgroups of a reduction kernel
static constexpr int RED_NT = 256;

size_t reduce_work_size(int m) { return sizeof(cx<double>) * (size_t)RED_WG * (m < 1 ? 1 : m); }

static inline int nblk_of(long n, int b) { return (int)((n + b - 1) / b); }

template <class D, class S>
__global__ void k_convert(long n, const cx<S>* __restrict__ in, cx<D>* __restrict__ out) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        out[e] = ccast<D>(in[e]);
}
template <class T>
__global__ void k_axpy(long n, cx<double> a, const cx<T>* __restrict__ x, cx<T>* __restrict__ y) {
    cx<T> at = ccast<T>(a);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) y[e] += at * x[e];
}
template <class T>
__global__ void k_xpay(long n, const cx<T>* __restrict__ x, cx<double> a, cx<T>* __restrict__ y) {
    cx<T> at = ccast<T>(a);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) y[e] = x[e] + at * y[e];
}
template <class T>
__global__ void k_scale(long n, cx<double> a, cx<T>* __restrict__ x) {
    cx<T> at = ccast<T>(a);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) x[e] = at * x[e];
}
template <class T>
__global__ void k_sub(long n, const cx<T>* __restrict__ a, const cx<T>* __restrict__ b, cx<T>* __restrict__ out) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) out[e] = a[e] - b[e];
}

static inline int grid_for(long n) {
    long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

template <class D, class S>
void vec_convert(long n, const cx<S>* in, cx<D>* out, hipStream_t s) {
    k_convert<D, S><<<grid_for(n), 256, 0, s>>>(n, in, out);
}
template <class T>
void vec_axpy(long n, cx<double> a, const cx<T>* x, cx<T>* y, hipStream_t s) {
    k_axpy<T><<<grid_for(n), 256, 0, s>>>(n, a, x, y);
}
template <class T>
void vec_xpay(long n, const cx<T>* x, cx<double> a, cx<T>* y, hipStream_t s) {
    k_xpay<T><<<grid_for(n), 256, 0, s>>>(n, x, a, y);
}
template <class T>
void vec_scale(long n, cx<double> a, cx<T>* x, hipStream_t s) {
    k_scale<T><<<grid_for(n), 256, 0, s>>>(n, a, x);
}
template <class T>
void vec_sub(long n, const cx<T>* a, const cx<T>* b, cx<T>* out, hipStream_t s) {
    k_sub<T><<<grid_for(n), 256, 0, s>>>(n, a, b, out);
}

// ---- last-workgroup reduction of m complex partials -----------------------
__device__ __forceinline__ void finish_partials(int m, cx<double>* part, int* count, cx<double>* out, bool add_to_out) {
    __shared__ int last;
    __threadfence();
    if (threadIdx.x == 0) last = (atomicAdd(count, 1) == (int)gridDim.x - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        cx<double> s = czero<double>();
        for (int b = 0; b < (int)gridDim.x; b++) s += part[(size_t)b * m + i];
        out[i] = s;
    }
    if (threadIdx.x == 0) *count = 0;
    (void)add_to_out;
}

template <class T>
__global__ void __launch_bounds__(RED_NT) k_multidot(long n, int m, const cx<T>* __restrict__ V, long ldv,
                                                     const cx<T>* __restrict__ w, cx<double>* __restrict__ out,
                                                     cx<double>* part, int* count) {
    __shared__ cx<double> red[(RED_NT / 64) * MAXM];
    cx<double> acc[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; i++) acc[i] = czero<double>();
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        cx<double> we = ccast<double>(w[e]);
#pragma unroll
        for (int i = 0; i < MAXM; i++)
            if (i < m) acc[i] += cmulc(ccast<double>(V[(size_t)i * ldv + e]), we);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < MAXM; i++) {
        if (i < m) {
            double re = wave_sum(acc[i].re), im = wave_sum(acc[i].im);
            if (lane == 0) red[wv * MAXM + i] = {re, im};
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        cx<double> s = czero<double>();
        for (int q = 0; q < nw; q++) s += red[q * MAXM + i];
        part[(size_t)blockIdx.x * m + i] = s;
    }
    finish_partials(m, part, count, out, false);
}

template <class T>
__global__ void __launch_bounds__(RED_NT) k_update_norm(long n, int m, const cx<T>* __restrict__ V, long ldv,
                                                        const cx<double>* __restrict__ h, cx<T>* __restrict__ w,
                                                        cx<double>* __restrict__ out, cx<double>* part, int* count) {
    __shared__ cx<double> red[RED_NT / 64];
    cx<T> hh[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; i++) hh[i] = (i < m) ? ccast<T>(h[i]) : czero<T>();
    double acc = 0;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        cx<T> we = w[e];
#pragma unroll
        for (int i = 0; i < MAXM; i++)
            if (i < m) we -= hh[i] * V[(size_t)i * ldv + e];
        w[e] = we;
        acc += (double)norm2(we);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    acc = wave_sum(acc);
    if (lane == 0) red[wv] = {acc, 0.0};
    __syncthreads();
    if (threadIdx.x == 0) {
        cx<double> s = czero<double>();
        for (int q = 0; q < nw; q++) s += red[q];
        part[blockIdx.x] = s;
    }
    finish_partials(1, part, count, out, false);
}

template <class T>
void vec_multidot(long n, int m, const cx<T>* V, long ldv, const cx<T>* w, cx<double>* out, void* work, int* count,
                  hipStream_t s) {
    int nb = nblk_of(n, RED_NT);
    if (nb > RED_WG) nb = RED_WG;
    for (int i0 = 0; i0 < m; i0 += MAXM) {
        int mm = (m - i0 < MAXM) ? m - i0 : MAXM;
        k_multidot<T><<<nb, RED_NT, 0, s>>>(n, mm, V + (size_t)i0 * ldv, ldv, w, out + i0, (cx<double>*)work, count);
    }
}

template <class T>
void vec_update_norm(long n, int m, const cx<T>* V, long ldv, const cx<double>* h, cx<T>* w, cx<double>* out,
                     void* work, int* count, hipStream_t s) {
    int nb = nblk_of(n, RED_NT);
    if (nb > RED_WG) nb = RED_WG;
    // chunks of MAXM basis vectors: all but the last chunk only subtract
    int i0 = 0;
    while (m - i0 > MAXM) {
        k_update_norm<T><<<nb, RED_NT, 0, s>>>(n, MAXM, V + (size_t)i0 * ldv, ldv, h + i0, w, out, (cx<double>*)work, count);
        i0 += MAXM;
    }
    k_update_norm<T><<<nb, RED_NT, 0, s>>>(n, m - i0, V + (size_t)i0 * ldv, ldv, h + i0, w, out, (cx<double>*)work, count);
}

template <class T, class X>
__global__ void k_lincomb(long n, int m, const cx<T>* __restrict__ Z, long ldz, const cx<double>* __restrict__ y,
                          cx<X>* __restrict__ x) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        cx<double> s = ccast<double>(x[e]);
        for (int i = 0; i < m; i++) s += y[i] * ccast<double>(Z[(size_t)i * ldz + e]);
        x[e] = ccast<X>(s);
    }
}

template <class T, class X>
void vec_lincomb(long n, int m, const cx<T>* Z, long ldz, const cx<double>* y, cx<X>* x, hipStream_t s) {
    k_lincomb<T, X><<<grid_for(n), 256, 0, s>>>(n, m, Z, ldz, y, x);
}

template <class T>
__global__ void k_finite(long n, const cx<T>* __restrict__ x, int* bad) {
    int b = 0;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        if (!isfinite((double)x[e].re) || !isfinite((double)x[e].im)) b = 1;
    if (b) atomicOr(bad, 1);
}
template <class T>
void vec_finite_check(long n, const cx<T>* x, int* bad, hipStream_t s) {
    k_finite<T><<<grid_for(n), 256, 0, s>>>(n, x, bad);
}

#define DD_BLAS_INST(T)                                                                                            \
    template void vec_axpy<T>(long, cx<double>, const cx<T>*, cx<T>*, hipStream_t);                                \
    template void vec_xpay<T>(long, const cx<T>*, cx<double>, cx<T>*, hipStream_t);                                \
    template void vec_scale<T>(long, cx<double>, cx<T>*, hipStream_t);                                             \
    template void vec_sub<T>(long, const cx<T>*, const cx<T>*, cx<T>*, hipStream_t);                               \
    template void vec_multidot<T>(long, int, const cx<T>*, long, const cx<T>*, cx<double>*, void*, int*, hipStream_t); \
    template void vec_update_norm<T>(long, int, const cx<T>*, long, const cx<double>*, cx<T>*, cx<double>*, void*, int*, \
                                     hipStream_t);                                                                 \
    template void vec_finite_check<T>(long, const cx<T>*, int*, hipStream_t);

DD_BLAS_INST(double)
DD_BLAS_INST(float)
template void vec_convert<double, float>(long, const cx<float>*, cx<double>*, hipStream_t);
template void vec_convert<float, double>(long, const cx<double>*, cx<float>*, hipStream_t);
template void vec_convert<double, double>(long, const cx<double>*, cx<double>*, hipStream_t);
template void vec_convert<float, float>(long, const cx<float>*, cx<float>*, hipStream_t);
template void vec_lincomb<double, double>(long, int, const cx<double>*, long, const cx<double>*, cx<double>*, hipStream_t);
template void vec_lincomb<float, double>(long, int, const cx<float>*, long, const cx<double>*, cx<double>*, hipStream_t);
template void vec_lincomb<float, float>(long, int, const cx<float>*, long, const cx<double>*, cx<float>*, hipStream_t);

}  // namespace dd
