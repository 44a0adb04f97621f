// dd_blas.hip -- vector algebra for the Krylov solvers (FGMRES / GMRES).
//
// The Arnoldi step needs the inner products V_i^H w of one new vector against
// all basis vectors, then w -= V h and ||w||.  Accumulation is FP64 for every
// storage precision; partial sums are combined in a fixed order.
#include <algorithm>

#include "dd_kernels.h"

namespace dd {

static constexpr int MAXM = 32;        // basis vectors handled per launch
static constexpr int RED_CHUNKS = 1024;  // chunks a reduced vector is cut into
static constexpr int RED_NT = 256;
static constexpr int UN_BATCH = 16;    // basis vectors loaded together in k_update_norm
static_assert(RED_NT % MAXM == 0, "k_update_norm splits its threads into groups of MAXM");

size_t reduce_work_size(int m, int nr) {
    (void)m;
    // multidot partials, norm partials, and the partials of the fused update + inner products
    return sizeof(cx<double>) * (size_t)RED_CHUNKS * (2 * MAXM + 1) * (size_t)(nr < 1 ? 1 : nr);
}

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

static inline dim3 grid_b(long n, int nr) {
    long b = (n + 255) / 256;
    long cap = 4096 / (nr < 1 ? 1 : nr);
    if (cap < 64) cap = 64;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return dim3((unsigned)b, (unsigned)(nr < 1 ? 1 : nr));
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
// The vector is cut into at most RED_CHUNKS chunks of at least 1024 entries.  multidot runs one
// workgroup per (chunk, basis vector, right-hand side) and writes the chunk's
// partial inner product; update_norm runs one workgroup per (chunk, RHS).  A
// small kernel then adds the partials in chunk order, so the results do not
// depend on scheduling.
static inline int red_chunks(long n) {
    // at least 1024 entries per chunk: every workgroup of update_norm first adds
    // all nc chunk partials of the inner products, a dependent chain of nc / 8
    // loads per thread, so short vectors want few chunks
    long c = (n + 1023) / 1024;
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

// part[(r*nc + c)*m + i] = chunk c of V_i^H w for RHS r
template <class T>
__global__ void __launch_bounds__(RED_NT) k_multidot(long n, long chunk, int nc, int m, const cx<T>* __restrict__ V,
                                                     long ldv, const cx<T>* __restrict__ w, cx<double>* __restrict__ part,
                                                     long ldr, long ldw, Mask mk) {
    const int c = blockIdx.x, i = blockIdx.y, r = blockIdx.z;
    if (!mk.on(r)) return;
    __shared__ double sh[2][RED_NT / 64];
    const long e0 = c * chunk, e1 = (e0 + chunk < n) ? e0 + chunk : n;
    const cx<T>* v = V + r * ldr + (size_t)i * ldv;
    const cx<T>* ww = w + r * ldw;
    double re = 0, im = 0;
    for (long e = e0 + threadIdx.x; e < e1; e += RED_NT) {
        cx<T> a = v[e], b = ww[e];
        re += (double)a.re * b.re + (double)a.im * b.im;
        im += (double)a.re * b.im - (double)a.im * b.re;
    }
    re = block_sum256(re, sh[0]);
    im = block_sum256(im, sh[1]);
    if (threadIdx.x == 0) part[((size_t)r * nc + c) * m + i] = cx<double>{re, im};
}

// out[r*ostride + i] = sum_c part[(r*nc + c)*m + i]; one workgroup per (i, r)
__global__ void __launch_bounds__(RED_NT) k_final_sum(int nc, int m, const cx<double>* __restrict__ part,
                                                      cx<double>* __restrict__ out, int ostride, Mask mk) {
    const int i = blockIdx.x, r = blockIdx.y;
    if (!mk.on(r)) return;
    __shared__ double sh[2][RED_NT / 64];
    double re = 0, im = 0;
    for (int c = threadIdx.x; c < nc; c += RED_NT) {
        cx<double> v = part[((size_t)r * nc + c) * m + i];
        re += v.re;
        im += v.im;
    }
    re = block_sum256(re, sh[0]);
    im = block_sum256(im, sh[1]);
    if (threadIdx.x == 0) out[(size_t)r * ostride + i] = cx<double>{re, im};
}

// w -= sum_i h_i V_i ; npart[r*nc + c] = chunk c of ||w||^2.  With hpart != 0
// the inner products are first summed from the multidot partials.
//
// With ga.st (the coarsest GMRES) the stored basis vectors may carry factors
// sc_i (V_i = sc_i * stored): the partial sums are of the stored vectors, so
// h_i = sc_i * sum and w -= sum_i (h_i sc_i) stored_i.  The last workgroup of
// each RHS to finish (atomic count in ga.done, reset by it) then adds the norm
// partials and folds the column into the state (and scales w when
// ga.normalize): the norm sum and the Givens update need no launch of their own.
struct GivensArgs {
    GmDev* st = nullptr;
    int j = 0;
    int* done = nullptr;
    int normalize = 0;
};
__device__ double gm_column_wg(GmDev* st, int j, const cx<double>* h, double hn2, bool normalize);

template <class T>
__global__ void __launch_bounds__(RED_NT) k_update_norm(long n, long chunk, int nc, int m, const cx<T>* __restrict__ V,
                                                        long ldv, const cx<double>* __restrict__ h, int hstride,
                                                        const cx<double>* __restrict__ hpart, cx<double>* hout,
                                                        cx<T>* __restrict__ w, cx<double>* __restrict__ npart, long ldr,
                                                        long ldw, Mask mk, GivensArgs ga, const double* __restrict__ g,
                                                        int gstride, cx<float>* __restrict__ wc, long ldc) {
    const int c = blockIdx.x, r = blockIdx.y;
    if (!mk.on(r)) return;
    const double* scv = ga.st ? ga.st[r].sc : nullptr;
    __shared__ double sh[RED_NT / 64];
    __shared__ cx<T> hh[MAXM];
    if (hpart) {
        // inner product i = sum over the chunk partials: thread (g, i) adds the
        // chunks c = g mod HG, then thread i adds the HG group sums (fixed order)
        constexpr int HG = RED_NT / MAXM;
        __shared__ cx<double> hg[HG][MAXM];
        const int i = threadIdx.x % MAXM, gq = threadIdx.x / MAXM;
        if (i < m) {
            cx<double> hv = czero<double>();
            for (int q = gq; q < nc; q += HG) hv += hpart[((size_t)r * nc + q) * m + i];
            hg[gq][i] = hv;
        }
        __syncthreads();
        if (threadIdx.x < m) {
            cx<double> hv = hg[0][threadIdx.x];
            for (int q = 1; q < HG; q++) hv += hg[q][threadIdx.x];
            const double f = scv ? scv[threadIdx.x] : 1.0;
            hv = f * hv;
            if (c == 0) hout[(size_t)r * hstride + threadIdx.x] = hv;
            hh[threadIdx.x] = ccast<T>(f * hv);
        }
    } else if (threadIdx.x < m) {
        const double gi = g ? g[(size_t)r * gstride + threadIdx.x] : 1.0;
        hh[threadIdx.x] = ccast<T>(gi * h[(size_t)r * hstride + threadIdx.x]);
    }
    __syncthreads();
    const cx<T>* Vr = V + r * ldr;
    cx<T>* wr = w + r * ldw;
    cx<float>* wcr = wc ? wc + r * ldc : nullptr;
    const long e0 = c * chunk, e1 = (e0 + chunk < n) ? e0 + chunk : n;
    double acc = 0;
    for (long e = e0 + threadIdx.x; e < e1; e += RED_NT) {
        cx<T> we = wr[e];
        // basis entries are loaded in batches so that many loads are in flight
        // (short coarse vectors leave one element per thread: latency bound)
        for (int i0 = 0; i0 < m; i0 += UN_BATCH) {
            cx<T> vv[UN_BATCH];
#pragma unroll
            for (int u = 0; u < UN_BATCH; u++) vv[u] = (i0 + u < m) ? Vr[(size_t)(i0 + u) * ldv + e] : czero<T>();
#pragma unroll
            for (int u = 0; u < UN_BATCH; u++)
                if (i0 + u < m) we -= hh[i0 + u] * vv[u];
        }
        wr[e] = we;
        if (wcr) wcr[e] = ccast<float>(we);
        acc += (double)norm2(we);
    }
    acc = block_sum256(acc, sh);
    if (threadIdx.x == 0) npart[(size_t)r * nc + c] = cx<double>{acc, 0.0};
    if (!ga.st) return;
    // ---- last workgroup of this RHS: norm, Givens update, next basis vector ----
    __shared__ int last_s;
    __threadfence();   // this workgroup's w entries, h (chunk 0) and norm partial
    if (threadIdx.x == 0) last_s = (atomicAdd(ga.done + r, 1) == nc - 1);
    __syncthreads();
    if (!last_s) return;
    __threadfence();
    double n2 = 0;
    for (int q = threadIdx.x; q < nc; q += RED_NT) n2 += npart[(size_t)r * nc + q].re;
    __syncthreads();   // sh is reused
    n2 = block_sum256(n2, sh);
    cx<double>* hr = hout + (size_t)r * hstride;
    if (threadIdx.x == 0) {
        hr[33] = cx<double>{n2, 0.0};
        ga.done[r] = 0;
    }
    const double f = gm_column_wg(ga.st + r, ga.j, hr, n2, ga.normalize != 0);
    if (ga.normalize && f != 0.0) {
        const T ft = T(f);
        constexpr int B = 8;   // entries per thread in flight
        for (long q0 = threadIdx.x; q0 < n; q0 += (long)B * RED_NT) {
            cx<T> v[B];
#pragma unroll
            for (int u = 0; u < B; u++) {
                const long q = q0 + (long)u * RED_NT;
                v[u] = (q < n) ? wr[q] : czero<T>();
            }
#pragma unroll
            for (int u = 0; u < B; u++) {
                const long q = q0 + (long)u * RED_NT;
                if (q < n) wr[q] = ft * v[u];
            }
        }
    }
}

static inline cx<double>* hpart_of(void* work) { return (cx<double>*)work; }
static inline cx<double>* npart_of(void* work, int nr) {
    return (cx<double>*)work + (size_t)RED_CHUNKS * MAXM * (nr < 1 ? 1 : nr);
}
static inline cx<double>* upart_of(void* work, int nr) {
    return (cx<double>*)work + (size_t)RED_CHUNKS * (MAXM + 1) * (nr < 1 ? 1 : nr);
}

// The first projection of a classical Gram-Schmidt pass with its
// reorthogonalisation's inner products in the same sweep: w -= sum_i h_i V_i,
// then part[(r*nc + c)*m + i] = chunk c of V_i^H w (the updated w), each basis
// entry loaded once for both (m <= UD_MAX).
static constexpr int UD_MAX = 16;
template <class T, int JM>
__global__ void __launch_bounds__(RED_NT) k_update_dot(long n, long chunk, int nc, int m, const cx<T>* __restrict__ V,
                                                       long ldv, const cx<double>* __restrict__ h, int hstride,
                                                       cx<T>* __restrict__ w, cx<double>* __restrict__ part, long ldr,
                                                       long ldw, Mask mk, const double* __restrict__ g, int gstride) {
    const int c = blockIdx.x, r = blockIdx.y;
    if (!mk.on(r)) return;
    __shared__ cx<T> hh[JM];
    __shared__ double sh[2][RED_NT / 64];
    if (threadIdx.x < m) {
        const double gi = g ? g[(size_t)r * gstride + threadIdx.x] : 1.0;
        hh[threadIdx.x] = ccast<T>(gi * h[(size_t)r * hstride + threadIdx.x]);
    }
    __syncthreads();
    const cx<T>* Vr = V + r * ldr;
    cx<T>* wr = w + r * ldw;
    const long e0 = c * chunk, e1 = (e0 + chunk < n) ? e0 + chunk : n;
    double are[JM], aim[JM];
#pragma unroll
    for (int i = 0; i < JM; i++) are[i] = aim[i] = 0.0;
    for (long e = e0 + threadIdx.x; e < e1; e += RED_NT) {
        cx<T> we = wr[e];
        cx<T> vv[JM];
#pragma unroll
        for (int i = 0; i < JM; i++) vv[i] = (i < m) ? Vr[(size_t)i * ldv + e] : czero<T>();
#pragma unroll
        for (int i = 0; i < JM; i++)
            if (i < m) we -= hh[i] * vv[i];
        wr[e] = we;
#pragma unroll
        for (int i = 0; i < JM; i++) {
            are[i] += (double)vv[i].re * we.re + (double)vv[i].im * we.im;
            aim[i] += (double)vv[i].re * we.im - (double)vv[i].im * we.re;
        }
    }
    for (int i = 0; i < m; i++) {
        const double a = block_sum256(are[i], sh[0]);
        const double b = block_sum256(aim[i], sh[1]);
        if (threadIdx.x == 0) part[((size_t)r * nc + c) * m + i] = cx<double>{a, b};
        __syncthreads();   // sh is reused by the next pair of sums
    }
}

template <class T>
void vec_multidot(long n, int m, const cx<T>* V, long ldv, const cx<T>* w, cx<double>* out, void* work, int* count,
                  hipStream_t s, RedBatch rb) {
    (void)count;
    const int nc = red_chunks(n);
    const long chunk = (n + nc - 1) / nc;
    for (int i0 = 0; i0 < m; i0 += MAXM) {
        int mm = (m - i0 < MAXM) ? m - i0 : MAXM;
        dim3 grid(nc, mm, rb.nr);
        k_multidot<T><<<grid, RED_NT, 0, s>>>(n, chunk, nc, mm, V + (size_t)i0 * ldv, ldv, w, hpart_of(work), rb.ldr,
                                              rb.ldw, rb.mk);
        dim3 g2(mm, rb.nr);
        k_final_sum<<<g2, RED_NT, 0, s>>>(nc, mm, hpart_of(work), out + i0, rb.ostride, rb.mk);
    }
}

template <class T>
bool vec_update_dot(long n, int m, const cx<T>* V, long ldv, const cx<double>* h, cx<T>* w, cx<double>* out,
                    void* work, hipStream_t s, RedBatch rb, const double* g, int gstride) {
    if (m > UD_MAX) return false;
    const int nc = red_chunks(n);
    const long chunk = (n + nc - 1) / nc;
    dim3 grid(nc, rb.nr);
    if (m <= 8)
        k_update_dot<T, 8><<<grid, RED_NT, 0, s>>>(n, chunk, nc, m, V, ldv, h, rb.ostride, w, upart_of(work, rb.nr),
                                                  rb.ldr, rb.ldw, rb.mk, g, gstride);
    else
        k_update_dot<T, UD_MAX><<<grid, RED_NT, 0, s>>>(n, chunk, nc, m, V, ldv, h, rb.ostride, w,
                                                       upart_of(work, rb.nr), rb.ldr, rb.ldw, rb.mk, g, gstride);
    dim3 g2(m, rb.nr);
    k_final_sum<<<g2, RED_NT, 0, s>>>(nc, m, upart_of(work, rb.nr), out, rb.ostride, rb.mk);
    return true;
}

template <class T>
void vec_update_norm(long n, int m, const cx<T>* V, long ldv, const cx<double>* h, cx<T>* w, cx<double>* out,
                     void* work, int* count, hipStream_t s, RedBatch rb, const double* g, int gstride, cx<float>* wc,
                     long ldc) {
    (void)count;
    const int nc = red_chunks(n);
    const long chunk = (n + nc - 1) / nc;
    int i0 = 0;
    do {
        int mm = (m - i0 < MAXM) ? m - i0 : MAXM;
        dim3 grid(nc, rb.nr);
        // the FP32 copy is written by the launch that leaves w final
        const bool last = i0 + mm >= m;
        k_update_norm<T><<<grid, RED_NT, 0, s>>>(n, chunk, nc, mm, V + (size_t)i0 * ldv, ldv, h + i0, rb.ostride, nullptr,
                                                 nullptr, w, npart_of(work, rb.nr), rb.ldr, rb.ldw, rb.mk, GivensArgs{},
                                                 g ? g + i0 : nullptr, gstride, last ? wc : nullptr, ldc);
        i0 += mm;
    } while (i0 < m);
    dim3 g2(1, rb.nr);
    k_final_sum<<<g2, RED_NT, 0, s>>>(nc, 1, npart_of(work, rb.nr), out, rb.ostride, rb.mk);
}

// ---- device-resident GMRES bookkeeping (one state per right-hand side) -----
__global__ void k_gm_start(GmDev* st0, const cx<double>* res, int rstride, double tol, int first, int m, int maxit,
                           int fixed, Mask mk) {
    GmDev* st = st0 + blockIdx.x;
    __shared__ int reset_s;
    __shared__ double beta_s;
    if (threadIdx.x == 0) {
        reset_s = 0;
        if (first) {
            st->its = 0;
            st->stop = 0;
            st->m = m;
            st->maxit = maxit;
            st->fixed = fixed;
        }
        // a right-hand side outside the batch's mask, or one that stopped in an
        // earlier cycle, contributes nothing to this cycle (j = 0)
        if (!mk.on(blockIdx.x)) {
            st->stop = 1;
            st->j = 0;
            st->scale = 0.0;
        } else if (!first && st->stop) {
            st->j = 0;
        } else {
            const double beta = sqrt(res[(size_t)blockIdx.x * rstride].re);
            if (first) st->tol_abs = tol * beta;
            st->j = 0;
            st->scale = (beta > 0) ? 1.0 / beta : 0.0;
            if (beta == 0.0) st->stop = 1;
            beta_s = beta;
            reset_s = 1;
        }
    }
    __syncthreads();
    if (!reset_s) return;
    // cleared by the whole workgroup (one thread would wait on a thousand stores);
    // v_0 is normalised explicitly (sc[0] = 1)
    for (int e = threadIdx.x; e < 33 * 32; e += blockDim.x) st->H[e] = czero<double>();
    for (int e = threadIdx.x; e < 33; e += blockDim.x) {
        st->g[e] = (e == 0) ? cx<double>{beta_s, 0.0} : czero<double>();
        st->sc[e] = 1.0;
    }
}

__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
    double d = norm2(b);
    return cx<double>{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// fold column j (inner products h[0..j], ||w||^2 = hn2) into the state of
// one RHS, by a whole workgroup (at least 32 threads): the inner
// products and the previous rotations are first staged in LDS by many
// threads at once, then one thread runs the rotation chain with the running
// entry in registers (the global-memory form waits on one load per rotation)
// Returns, in every thread, the factor that normalises the new basis vector
// (0 when this RHS stopped at this step: the vector is then left as it is).
__device__ double gm_column_wg(GmDev* st, int j, const cx<double>* h, double hn2, bool normalize) {
    __shared__ cx<double> hs[33], css[32], sns[32];
    __shared__ double sc_s;
    const int t = threadIdx.x;
    if (t <= j) hs[t] = h[t];
    if (t < j) {
        css[t] = st->cs[t];
        sns[t] = st->sn[t];
    }
    __syncthreads();
    if (t == 0) {
        cx<double>* col = st->H + (size_t)j * 33;
        const double hn = sqrt(hn2);
        cx<double> a = hs[0];
        for (int i = 0; i < j; i++) {  // previous rotations; col[i] is final after rotation i
            const cx<double> b = hs[i + 1];
            col[i] = conj(css[i]) * a + conj(sns[i]) * b;
            a = -(sns[i] * a) + css[i] * b;
        }
        const cx<double> b = cx<double>{hn, 0.0};
        const double den = sqrt(norm2(a) + norm2(b));
        cx<double> c, s;
        if (den == 0.0) { c = cx<double>{1.0, 0.0}; s = czero<double>(); }
        else { c = cx<double>{a.re / den, a.im / den}; s = cx<double>{b.re / den, b.im / den}; }
        st->cs[j] = c;
        st->sn[j] = s;
        col[j] = conj(c) * a + conj(s) * b;
        col[j + 1] = czero<double>();
        const cx<double> gj = st->g[j];
        st->g[j + 1] = -(s * gj);
        st->g[j] = conj(c) * gj;
        st->its += 1;
        st->j = j + 1;
        const double resid = sqrt(norm2(st->g[j + 1]));
        int stop = 0;
        if (st->fixed > 0) stop = st->its >= st->fixed;
        else stop = (resid <= st->tol_abs) || (st->its >= st->maxit);
        if (hn == 0.0) stop = 1;
        st->stop = stop;
        st->scale = (hn > 0) ? 1.0 / hn : 0.0;
        // the new basis vector: w scaled by the caller (normalize), or w kept
        // with its factor
        st->sc[j + 1] = normalize ? 1.0 : st->scale;
        sc_s = stop ? 0.0 : st->scale;
    }
    __syncthreads();
    return sc_s;
}

// back substitution R y = g with the rotated Hessenberg R (k x k upper
// triangle), by columns: once y_i is known every thread r < i removes
// R_ri y_i from its g_r.  R and g are staged in LDS first (at least 32 threads).
__global__ void k_gm_solve(GmDev* st0) {
    GmDev* st = st0 + blockIdx.x;
    __shared__ cx<double> Rs[32 * 33], gsh[33], ys[32];
    const int k = st->j, t = threadIdx.x;
    for (int e = t; e < k * 33; e += blockDim.x) Rs[e] = st->H[e];
    for (int e = t; e < k; e += blockDim.x) gsh[e] = st->g[e];
    __syncthreads();
    for (int i = k - 1; i >= 0; i--) {
        if (t == 0) ys[i] = cdiv(gsh[i], Rs[i * 33 + i]);
        __syncthreads();
        if (t < i) gsh[t] -= Rs[i * 33 + t] * ys[i];
        __syncthreads();
    }
    for (int e = t; e < k; e += blockDim.x) st->y[e] = ys[e];
}

void gm_start(GmDev* st, const cx<double>* res, int rstride, double tol, int first, int m, int maxit, int fixed,
              int nr, hipStream_t s, Mask mk) {
    k_gm_start<<<nr, 64, 0, s>>>(st, res, rstride, tol, first, m, maxit, fixed, mk);
}

__global__ void k_gm_gather(const GmDev* st, int nr, int* out) {
    const int r = threadIdx.x;
    if (r < nr) {
        out[3 * r] = st[r].j;
        out[3 * r + 1] = st[r].its;
        out[3 * r + 2] = st[r].stop;
    }
}
void gm_gather(const GmDev* st, int nr, int* out, hipStream_t s) { k_gm_gather<<<1, 64, 0, s>>>(st, nr, out); }
void gm_solve(GmDev* st, int nr, hipStream_t s) { k_gm_solve<<<nr, 64, 0, s>>>(st); }

template <class T>
__global__ void k_scale_dev(long n, const GmDev* st0, cx<T>* __restrict__ x, const cx<T>* src, int ignore_stop,
                            long ld) {
    const GmDev* st = st0 + blockIdx.y;
    if (!ignore_stop && st->stop) return;
    x += blockIdx.y * ld;
    const cx<T>* in = src ? src + blockIdx.y * ld : x;
    const T sc = T(st->scale);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) x[e] = sc * in[e];
}
template <class T>
void vec_scale_dev(long n, const GmDev* st, cx<T>* x, hipStream_t s, bool ignore_stop, int nr, long ld,
                   const cx<T>* src) {
    dim3 grid(grid_for(n), nr);
    k_scale_dev<T><<<grid, 256, 0, s>>>(n, st, x, src, ignore_stop ? 1 : 0, ld);
}

template <class T>
__global__ void k_lincomb_dev(long n, const cx<T>* __restrict__ V, long ldv, const GmDev* st0, cx<T>* __restrict__ x,
                              long ldr, long ldx, int assign) {
    const GmDev* st = st0 + blockIdx.y;
    const int m = st->j;
    V += blockIdx.y * ldr;
    x += blockIdx.y * ldx;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        cx<double> sacc = assign ? czero<double>() : ccast<double>(x[e]);
        for (int i = 0; i < m; i++) sacc += st->y[i] * (st->sc[i] * ccast<double>(V[(size_t)i * ldv + e]));
        x[e] = ccast<T>(sacc);
    }
}
template <class T>
void vec_lincomb_dev(long n, const cx<T>* V, long ldv, const GmDev* st, cx<T>* x, hipStream_t s, int nr, long ldr,
                     long ldx, bool assign) {
    dim3 grid(grid_for(n), nr);
    k_lincomb_dev<T><<<grid, 256, 0, s>>>(n, V, ldv, st, x, ldr, ldx, assign ? 1 : 0);
}

template <class T>
void vec_multidot_skip(long n, int m, const cx<T>* V, long ldv, const cx<T>* w, void* work, hipStream_t s,
                       RedBatch rb) {
    const int nc = red_chunks(n);
    const long chunk = (n + nc - 1) / nc;
    dim3 grid(nc, m, rb.nr);
    k_multidot<T><<<grid, RED_NT, 0, s>>>(n, chunk, nc, m, V, ldv, w, hpart_of(work), rb.ldr, rb.ldw, rb.mk);
}

template <class T>
void vec_update_norm_givens(long n, int m, const cx<T>* V, long ldv, cx<T>* w, cx<double>* res, void* work,
                            hipStream_t s, RedBatch rb, GmDev* st, int j, int* done, bool normalize) {
    const int nc = red_chunks(n);
    const long chunk = (n + nc - 1) / nc;
    dim3 grid(nc, rb.nr);
    k_update_norm<T><<<grid, RED_NT, 0, s>>>(n, chunk, nc, m, V, ldv, nullptr, rb.ostride, hpart_of(work), res, w,
                                             npart_of(work, rb.nr), rb.ldr, rb.ldw, rb.mk,
                                             GivensArgs{st, j, done, normalize ? 1 : 0}, nullptr, 0, nullptr, 0);
}

template <class T, class X>
__global__ void k_lincomb(long n, Counts mc, const cx<T>* __restrict__ Z, long ldz, const cx<double>* __restrict__ y,
                          cx<X>* __restrict__ x, long ldzr, int ystride, long ldx, Mask mk) {
    if (!mk.on(blockIdx.y)) return;
    const int m = mc.v[blockIdx.y];
    Z += blockIdx.y * ldzr;
    y += (size_t)blockIdx.y * ystride;
    x += blockIdx.y * ldx;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        cx<double> sacc = ccast<double>(x[e]);
        for (int i = 0; i < m; i++) sacc += y[i] * ccast<double>(Z[(size_t)i * ldz + e]);
        x[e] = ccast<X>(sacc);
    }
}

template <class T, class X>
void vec_lincomb(long n, int m, const cx<T>* Z, long ldz, const cx<double>* y, cx<X>* x, hipStream_t s, int nr,
                 long ldzr, int ystride, long ldx, Mask mk, const Counts* per) {
    Counts mc;
    for (int r = 0; r < MAX_RHS; r++) mc.v[r] = (per && r < nr) ? std::min(per->v[r], m) : m;
    k_lincomb<T, X><<<grid_b(n, nr), 256, 0, s>>>(n, mc, Z, ldz, y, x, ldzr, ystride, ldx, mk);
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


// ---- batched element-wise operations (RHS r at base + r*ld, grid.y = RHS) --
template <class D, class S>
__global__ void k_convert_b(long n, const cx<S>* __restrict__ in, cx<D>* __restrict__ out, long ld, Mask mk) {
    if (!mk.on(blockIdx.y)) return;
    in += blockIdx.y * ld;
    out += blockIdx.y * ld;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        out[e] = ccast<D>(in[e]);
}
template <class T>
__global__ void k_sub_b(long n, const cx<T>* __restrict__ a, const cx<T>* __restrict__ b, cx<T>* __restrict__ out,
                        long ld, Mask mk) {
    if (!mk.on(blockIdx.y)) return;
    const long o = blockIdx.y * ld;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        out[o + e] = a[o + e] - b[o + e];
}
template <class T>
__global__ void k_scale_b(long n, Coefs c, cx<T>* __restrict__ x, long ld, Mask mk) {
    if (!mk.on(blockIdx.y)) return;
    x += blockIdx.y * ld;
    const T f = T(c.v[blockIdx.y]);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) x[e] = f * x[e];
}
// g[r * gstride + idx] = c.v[r] for the RHS the mask keeps
__global__ void k_set_factor(double* g, int gstride, int idx, Coefs c, int nr, Mask mk) {
    const int r = threadIdx.x;
    if (r < nr && mk.on(r)) g[(size_t)r * gstride + idx] = c.v[r];
}
void set_factor(double* g, int gstride, int idx, const Coefs& c, int nr, Mask mk, hipStream_t s) {
    k_set_factor<<<1, 64, 0, s>>>(g, gstride, idx, c, nr, mk);
}
__global__ void k_set_flags(int* d, unsigned bits, int n) {
    if ((int)threadIdx.x < n) d[threadIdx.x] = (bits >> threadIdx.x) & 1u;
}


template <class D, class S>
void bvec_convert(long n, const cx<S>* in, cx<D>* out, long ld, int nr, Mask mk, hipStream_t s) {
    k_convert_b<D, S><<<grid_b(n, nr), 256, 0, s>>>(n, in, out, ld, mk);
}
template <class T>
void bvec_sub(long n, const cx<T>* a, const cx<T>* b, cx<T>* out, long ld, int nr, Mask mk, hipStream_t s) {
    k_sub_b<T><<<grid_b(n, nr), 256, 0, s>>>(n, a, b, out, ld, mk);
}
template <class T>
void bvec_scale(long n, const Coefs& c, cx<T>* x, long ld, int nr, Mask mk, hipStream_t s) {
    k_scale_b<T><<<grid_b(n, nr), 256, 0, s>>>(n, c, x, ld, mk);
}
void set_flags(int* d, unsigned bits, int n, hipStream_t s) { k_set_flags<<<1, 64, 0, s>>>(d, bits, n); }

#define DD_BLAS_INST(T)                                                                                            \
    template void vec_axpy<T>(long, cx<double>, const cx<T>*, cx<T>*, hipStream_t);                                \
    template void vec_xpay<T>(long, const cx<T>*, cx<double>, cx<T>*, hipStream_t);                                \
    template void vec_scale<T>(long, cx<double>, cx<T>*, hipStream_t);                                             \
    template void vec_sub<T>(long, const cx<T>*, const cx<T>*, cx<T>*, hipStream_t);                               \
    template void vec_multidot<T>(long, int, const cx<T>*, long, const cx<T>*, cx<double>*, void*, int*, hipStream_t, \
                                  RedBatch);                                                                       \
    template bool vec_update_dot<T>(long, int, const cx<T>*, long, const cx<double>*, cx<T>*, cx<double>*, void*,       \
                                    hipStream_t, RedBatch, const double*, int);                                    \
    template void vec_update_norm<T>(long, int, const cx<T>*, long, const cx<double>*, cx<T>*, cx<double>*, void*, int*, \
                                     hipStream_t, RedBatch, const double*, int, cx<float>*, long);                 \
    template void vec_finite_check<T>(long, const cx<T>*, int*, hipStream_t);                                     \
    template void bvec_sub<T>(long, const cx<T>*, const cx<T>*, cx<T>*, long, int, Mask, hipStream_t);            \
    template void bvec_scale<T>(long, const Coefs&, cx<T>*, long, int, Mask, hipStream_t);                         \
    template void vec_scale_dev<T>(long, const GmDev*, cx<T>*, hipStream_t, bool, int, long, const cx<T>*);        \
    template void vec_lincomb_dev<T>(long, const cx<T>*, long, const GmDev*, cx<T>*, hipStream_t, int, long, long,  \
                                     bool);                                                                         \
    template void vec_multidot_skip<T>(long, int, const cx<T>*, long, const cx<T>*, void*, hipStream_t, RedBatch);  \
    template void vec_update_norm_givens<T>(long, int, const cx<T>*, long, cx<T>*, cx<double>*, void*, hipStream_t, \
                                            RedBatch, GmDev*, int, int*, bool);

DD_BLAS_INST(double)
DD_BLAS_INST(float)
template void vec_convert<double, float>(long, const cx<float>*, cx<double>*, hipStream_t);
template void vec_convert<float, double>(long, const cx<double>*, cx<float>*, hipStream_t);
template void vec_convert<double, double>(long, const cx<double>*, cx<double>*, hipStream_t);
template void vec_convert<float, float>(long, const cx<float>*, cx<float>*, hipStream_t);
template void vec_convert<_Float16, float>(long, const cx<float>*, cx<_Float16>*, hipStream_t);
template void bvec_convert<double, float>(long, const cx<float>*, cx<double>*, long, int, Mask, hipStream_t);
template void bvec_convert<float, double>(long, const cx<double>*, cx<float>*, long, int, Mask, hipStream_t);
template void bvec_convert<double, double>(long, const cx<double>*, cx<double>*, long, int, Mask, hipStream_t);
#define DD_LINCOMB_INST(T, X) \
    template void vec_lincomb<T, X>(long, int, const cx<T>*, long, const cx<double>*, cx<X>*, hipStream_t, int, long, int, long, Mask, \
                                    const Counts*);
DD_LINCOMB_INST(double, double)
DD_LINCOMB_INST(float, double)
DD_LINCOMB_INST(float, float)

}  // namespace dd
