// dd_blas.hip -- vector algebra for the Krylov solvers (FGMRES / GMRES).
//
// The Arnoldi step needs the inner products V_i^H w of one new vector against
// all basis vectors, then w -= V h and ||w||.  Accumulation is FP64 for every
// storage precision; partial sums are combined in a fixed order.
#include "dd_kernels.h"

namespace dd {

static constexpr int MAXM = 32;        // basis vectors handled per launch
static constexpr int RED_CHUNKS = 1024;  // chunks a reduced vector is cut into
static constexpr int RED_NT = 256;

size_t reduce_work_size(int m) { return sizeof(cx<double>) * (size_t)RED_CHUNKS * ((m < MAXM ? MAXM : m) + 1); }

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

// ---- reductions ------------------------------------------------------------
// The vector is cut into at most RED_CHUNKS chunks.  multidot runs one
// workgroup per (chunk, basis vector) and writes the chunk's partial inner
// product; update_norm runs one workgroup per chunk.  A one-workgroup kernel
// then adds the partials in chunk order, so the result does not depend on
// scheduling.
static inline int red_chunks(long n) {
    long c = (n + 255) / 256;
    if (c > RED_CHUNKS) c = RED_CHUNKS;
    if (c < 1) c = 1;
    return (int)c;
}

__device__ __forceinline__ double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); q++) s += sh[q];
    return s;
}

template <class T>
__global__ void __launch_bounds__(RED_NT) k_multidot(long n, long chunk, const cx<T>* __restrict__ V, long ldv,
                                                     const cx<T>* __restrict__ w, cx<double>* __restrict__ part, int m) {
    __shared__ double sh[2][RED_NT / 64];
    const int c = blockIdx.x, i = blockIdx.y;
    const long e0 = c * chunk, e1 = (e0 + chunk < n) ? e0 + chunk : n;
    const cx<T>* v = V + (size_t)i * ldv;
    double re = 0, im = 0;
    for (long e = e0 + threadIdx.x; e < e1; e += RED_NT) {
        cx<T> a = v[e], b = w[e];
        re += (double)a.re * b.re + (double)a.im * b.im;
        im += (double)a.re * b.im - (double)a.im * b.re;
    }
    re = block_sum256(re, sh[0]);
    im = block_sum256(im, sh[1]);
    if (threadIdx.x == 0) part[(size_t)c * m + i] = cx<double>{re, im};
}

// one workgroup per output: strided partial sums, then a fixed-shape tree
__global__ void __launch_bounds__(RED_NT) k_final_sum(int nchunk, int m, const cx<double>* __restrict__ part,
                                                      cx<double>* __restrict__ out) {
    __shared__ double sh[2][RED_NT / 64];
    const int i = blockIdx.x;
    double re = 0, im = 0;
    for (int c = threadIdx.x; c < nchunk; c += RED_NT) {
        cx<double> v = part[(size_t)c * m + i];
        re += v.re;
        im += v.im;
    }
    re = block_sum256(re, sh[0]);
    im = block_sum256(im, sh[1]);
    if (threadIdx.x == 0) out[i] = cx<double>{re, im};
}

template <class T>
__global__ void __launch_bounds__(RED_NT) k_update_norm(long n, long chunk, int m, const cx<T>* __restrict__ V, long ldv,
                                                        const cx<double>* __restrict__ h, cx<T>* __restrict__ w,
                                                        cx<double>* __restrict__ part) {
    __shared__ double sh[RED_NT / 64];
    __shared__ cx<T> hh[MAXM];
    if (threadIdx.x < m) hh[threadIdx.x] = ccast<T>(h[threadIdx.x]);
    __syncthreads();
    const int c = blockIdx.x;
    const long e0 = c * chunk, e1 = (e0 + chunk < n) ? e0 + chunk : n;
    double acc = 0;
    for (long e = e0 + threadIdx.x; e < e1; e += RED_NT) {
        cx<T> we = w[e];
        for (int i = 0; i < m; i++) we -= hh[i] * V[(size_t)i * ldv + e];
        w[e] = we;
        acc += (double)norm2(we);
    }
    acc = block_sum256(acc, sh);
    if (threadIdx.x == 0) part[c] = cx<double>{acc, 0.0};
}

template <class T>
void vec_multidot(long n, int m, const cx<T>* V, long ldv, const cx<T>* w, cx<double>* out, void* work, int* count,
                  hipStream_t s) {
    (void)count;
    const int nc = red_chunks(n);
    const long chunk = (n + nc - 1) / nc;
    for (int i0 = 0; i0 < m; i0 += MAXM) {
        int mm = (m - i0 < MAXM) ? m - i0 : MAXM;
        dim3 grid(nc, mm);
        k_multidot<T><<<grid, RED_NT, 0, s>>>(n, chunk, V + (size_t)i0 * ldv, ldv, w, (cx<double>*)work, mm);
        k_final_sum<<<mm, RED_NT, 0, s>>>(nc, mm, (const cx<double>*)work, out + i0);
    }
}

template <class T>
void vec_update_norm(long n, int m, const cx<T>* V, long ldv, const cx<double>* h, cx<T>* w, cx<double>* out,
                     void* work, int* count, hipStream_t s) {
    (void)count;
    const int nc = red_chunks(n);
    const long chunk = (n + nc - 1) / nc;
    int i0 = 0;
    do {
        int mm = (m - i0 < MAXM) ? m - i0 : MAXM;
        k_update_norm<T><<<nc, RED_NT, 0, s>>>(n, chunk, mm, V + (size_t)i0 * ldv, ldv, h + i0, w, (cx<double>*)work);
        i0 += mm;
    } while (i0 < m);
    k_final_sum<<<1, RED_NT, 0, s>>>(nc, 1, (const cx<double>*)work, out);
}

// ---- device-resident GMRES bookkeeping ------------------------------------
__global__ void k_gm_start(GmDev* st, const cx<double>* beta2, double tol, int first, int m, int maxit, int fixed) {
    if (threadIdx.x != 0) return;
    double beta = sqrt(beta2->re);
    if (first) {
        st->tol_abs = tol * beta;
        st->its = 0;
        st->stop = (beta == 0.0) ? 1 : 0;
        st->m = m;
        st->maxit = maxit;
        st->fixed = fixed;
    }
    for (int i = 0; i < 33; i++) st->g[i] = czero<double>();
    for (int i = 0; i < 33 * 32; i++) st->H[i] = czero<double>();
    st->g[0] = cx<double>{beta, 0.0};
    st->j = 0;
    st->scale = (beta > 0) ? 1.0 / beta : 0.0;
    if (beta == 0.0) st->stop = 1;
}

__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
    double d = norm2(b);
    return cx<double>{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

__global__ void k_gm_column(GmDev* st, int j, const cx<double>* __restrict__ h, const cx<double>* __restrict__ hn2) {
    if (threadIdx.x != 0 || st->stop) return;
    cx<double>* col = st->H + (size_t)j * 33;
    for (int i = 0; i <= j; i++) col[i] = h[i];
    double hn = sqrt(hn2->re);
    col[j + 1] = cx<double>{hn, 0.0};
    for (int i = 0; i < j; i++) {  // previous rotations
        cx<double> a = col[i], b = col[i + 1];
        col[i] = conj(st->cs[i]) * a + conj(st->sn[i]) * b;
        col[i + 1] = -(st->sn[i] * a) + st->cs[i] * b;
    }
    cx<double> a = col[j], b = col[j + 1];
    double den = sqrt(norm2(a) + norm2(b));
    if (den == 0.0) { st->cs[j] = cx<double>{1.0, 0.0}; st->sn[j] = czero<double>(); }
    else { st->cs[j] = cx<double>{a.re / den, a.im / den}; st->sn[j] = cx<double>{b.re / den, b.im / den}; }
    col[j] = conj(st->cs[j]) * a + conj(st->sn[j]) * b;
    col[j + 1] = czero<double>();
    st->g[j + 1] = -(st->sn[j] * st->g[j]);
    st->g[j] = conj(st->cs[j]) * st->g[j];
    st->its += 1;
    st->j = j + 1;
    double res = sqrt(norm2(st->g[j + 1]));
    int stop = 0;
    if (st->fixed > 0) stop = st->its >= st->fixed;
    else stop = (res <= st->tol_abs) || (st->its >= st->maxit);
    if (hn == 0.0) stop = 1;
    st->stop = stop;
    st->scale = (hn > 0) ? 1.0 / hn : 0.0;
}

__global__ void k_gm_solve(GmDev* st) {
    if (threadIdx.x != 0) return;
    int k = st->j;
    for (int i = k - 1; i >= 0; i--) {
        cx<double> sacc = st->g[i];
        for (int q = i + 1; q < k; q++) sacc -= st->H[(size_t)q * 33 + i] * st->y[q];
        st->y[i] = cdiv(sacc, st->H[(size_t)i * 33 + i]);
    }
}

void gm_start(GmDev* st, const cx<double>* beta2, double tol, int first, int m, int maxit, int fixed, hipStream_t s) {
    k_gm_start<<<1, 64, 0, s>>>(st, beta2, tol, first, m, maxit, fixed);
}
void gm_column(GmDev* st, int j, const cx<double>* h, const cx<double>* hn2, hipStream_t s) {
    k_gm_column<<<1, 64, 0, s>>>(st, j, h, hn2);
}
void gm_solve(GmDev* st, hipStream_t s) { k_gm_solve<<<1, 64, 0, s>>>(st); }

template <class T>
__global__ void k_scale_dev(long n, const GmDev* st, cx<T>* __restrict__ x, int ignore_stop) {
    if (!ignore_stop && st->stop) return;
    const T sc = T(st->scale);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) x[e] = sc * x[e];
}
template <class T>
void vec_scale_dev(long n, const GmDev* st, cx<T>* x, hipStream_t s, bool ignore_stop) {
    k_scale_dev<T><<<grid_for(n), 256, 0, s>>>(n, st, x, ignore_stop ? 1 : 0);
}

template <class T>
__global__ void k_lincomb_dev(long n, const cx<T>* __restrict__ V, long ldv, const GmDev* st, cx<T>* __restrict__ x) {
    const int m = st->j;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        cx<double> sacc = ccast<double>(x[e]);
        for (int i = 0; i < m; i++) sacc += st->y[i] * ccast<double>(V[(size_t)i * ldv + e]);
        x[e] = ccast<T>(sacc);
    }
}
template <class T>
void vec_lincomb_dev(long n, const cx<T>* V, long ldv, const GmDev* st, cx<T>* x, hipStream_t s) {
    k_lincomb_dev<T><<<grid_for(n), 256, 0, s>>>(n, V, ldv, st, x);
}

// skip-aware Arnoldi reductions: the multidot partials are summed by every
// workgroup of the update kernel itself (fixed order), saving a launch
template <class T>
__global__ void __launch_bounds__(RED_NT) k_multidot_skip(long n, long chunk, const cx<T>* __restrict__ V, long ldv,
                                                          const cx<T>* __restrict__ w, cx<double>* __restrict__ part,
                                                          int m, const int* skip) {
    if (*skip) return;
    __shared__ double sh[2][RED_NT / 64];
    const int c = blockIdx.x, i = blockIdx.y;
    const long e0 = c * chunk, e1 = (e0 + chunk < n) ? e0 + chunk : n;
    const cx<T>* v = V + (size_t)i * ldv;
    double re = 0, im = 0;
    for (long e = e0 + threadIdx.x; e < e1; e += RED_NT) {
        cx<T> a = v[e], b = w[e];
        re += (double)a.re * b.re + (double)a.im * b.im;
        im += (double)a.re * b.im - (double)a.im * b.re;
    }
    re = block_sum256(re, sh[0]);
    im = block_sum256(im, sh[1]);
    if (threadIdx.x == 0) part[(size_t)c * m + i] = cx<double>{re, im};
}

template <class T>
__global__ void __launch_bounds__(RED_NT) k_update_norm_skip(long n, long chunk, int nc, int m, const cx<T>* __restrict__ V,
                                                             long ldv, const cx<double>* __restrict__ hpart,
                                                             cx<T>* __restrict__ w, cx<double>* __restrict__ hout,
                                                             cx<double>* __restrict__ npart, const int* skip) {
    if (*skip) return;
    __shared__ double sh[RED_NT / 64];
    __shared__ cx<T> hh[MAXM];
    if (threadIdx.x < m) {
        cx<double> sacc = czero<double>();
        for (int c = 0; c < nc; c++) sacc += hpart[(size_t)c * m + threadIdx.x];
        hh[threadIdx.x] = ccast<T>(sacc);
        if (blockIdx.x == 0) hout[threadIdx.x] = sacc;
    }
    __syncthreads();
    const int c = blockIdx.x;
    const long e0 = c * chunk, e1 = (e0 + chunk < n) ? e0 + chunk : n;
    double acc = 0;
    for (long e = e0 + threadIdx.x; e < e1; e += RED_NT) {
        cx<T> we = w[e];
        for (int i = 0; i < m; i++) we -= hh[i] * V[(size_t)i * ldv + e];
        w[e] = we;
        acc += (double)norm2(we);
    }
    acc = block_sum256(acc, sh);
    if (threadIdx.x == 0) npart[c] = cx<double>{acc, 0.0};
}

__global__ void k_final_norm_skip(int nchunk, const cx<double>* __restrict__ part, cx<double>* __restrict__ out,
                                  const int* skip) {
    if (*skip) return;
    __shared__ double sh[RED_NT / 64];
    double re = 0;
    for (int c = threadIdx.x; c < nchunk; c += RED_NT) re += part[c].re;
    re = block_sum256(re, sh);
    if (threadIdx.x == 0) out[0] = cx<double>{re, 0.0};
}

// `out` receives h (m entries); `work` holds the multidot partials, followed
// by RED_CHUNKS norm partials
template <class T>
void vec_multidot_skip(long n, int m, const cx<T>* V, long ldv, const cx<T>* w, cx<double>* out, void* work,
                       const int* skip, hipStream_t s) {
    (void)out;
    const int nc = red_chunks(n);
    const long chunk = (n + nc - 1) / nc;
    dim3 grid(nc, m);
    k_multidot_skip<T><<<grid, RED_NT, 0, s>>>(n, chunk, V, ldv, w, (cx<double>*)work, m, skip);
}
template <class T>
void vec_update_norm_skip(long n, int m, const cx<T>* V, long ldv, const cx<double>* h, cx<T>* w, cx<double>* out,
                          void* work, const int* skip, hipStream_t s) {
    const int nc = red_chunks(n);
    const long chunk = (n + nc - 1) / nc;
    cx<double>* hpart = (cx<double>*)work;
    cx<double>* npart = hpart + (size_t)RED_CHUNKS * MAXM;
    k_update_norm_skip<T><<<nc, RED_NT, 0, s>>>(n, chunk, nc, m, V, ldv, hpart, w, const_cast<cx<double>*>(h), npart, skip);
    k_final_norm_skip<<<1, RED_NT, 0, s>>>(nc, npart, out, skip);
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
    template void vec_finite_check<T>(long, const cx<T>*, int*, hipStream_t);                                     \
    template void vec_scale_dev<T>(long, const GmDev*, cx<T>*, hipStream_t, bool);                                 \
    template void vec_lincomb_dev<T>(long, const cx<T>*, long, const GmDev*, cx<T>*, hipStream_t);                 \
    template void vec_multidot_skip<T>(long, int, const cx<T>*, long, const cx<T>*, cx<double>*, void*, const int*, \
                                       hipStream_t);                                                              \
    template void vec_update_norm_skip<T>(long, int, const cx<T>*, long, const cx<double>*, cx<T>*, cx<double>*, void*, \
                                          const int*, hipStream_t);

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
