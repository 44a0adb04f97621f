// dd_common.h -- device/host building blocks of the MI355X DD-alpha-AMG path:
// complex arithmetic, the even-odd block-major lattice layout, the spin
// structure of the chiral gamma matrices, packed Hermitian 6x6 clover blocks
// and wavefront/workgroup reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dd {

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <class T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <class T> __host__ __device__ __forceinline__ cx<T> mkc(T r, T i) { return cx<T>{r, i}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T>& operator+=(cx<T>& a, cx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <class T> __host__ __device__ __forceinline__ cx<T>& operator-=(cx<T>& a, cx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <class T> __host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <class T> __host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class T> __host__ __device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.im, a.re}; }
template <class T> __host__ __device__ __forceinline__ cx<T> times_mi(cx<T> a) { return {a.im, -a.re}; }
template <class T> __host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <class T> __host__ __device__ __forceinline__ cx<T> czero() { return {T(0), T(0)}; }
template <class D, class S> __host__ __device__ __forceinline__ cx<D> ccast(cx<S> a) { return {D(a.re), D(a.im)}; }
// fused multiply-add; acc += a b and acc += conj(a) b as four of them (written
// out: the compiler does not contract a sum of products into an accumulator)
__host__ __device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <class T> __host__ __device__ __forceinline__ void cmac(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.re = fmadd(a.re, b.re, acc.re);
    acc.re = fmadd(-a.im, b.im, acc.re);
    acc.im = fmadd(a.re, b.im, acc.im);
    acc.im = fmadd(a.im, b.re, acc.im);
}
template <class T> __host__ __device__ __forceinline__ void cmacc(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.re = fmadd(a.re, b.re, acc.re);
    acc.re = fmadd(a.im, b.im, acc.re);
    acc.im = fmadd(a.re, b.im, acc.im);
    acc.im = fmadd(-a.im, b.re, acc.im);
}

// FP16 storage of fine-level spinor sets with one FP32 scale per (parity,
// chirality half, site).  Per site and half (p, h) seven 4-byte slots at
// d[((2p + h) 7 + c) vh + i]: for c < 6 the entry 6h + c of the spinor
// (real and imaginary part in FP16, divided by the scale), for c = 6 the
// scale itself (FP32 bits: the largest modulus of the half's 12 reals, so the
// stored values lie in [-1, 1]).  A set of n = 24 vh complex entries takes
// 28 vh slots; an offset of `off` complex entries (a multiple of 6 vh, e.g.
// one vector) is 7 off / 6 slots.
typedef _Float16 hpair __attribute__((ext_vector_type(2)));
struct hspin {
    hpair* d;
    __host__ __device__ __forceinline__ hspin operator+(long off) const { return hspin{d + off / 6 * 7}; }
};


// ---------------------------------------------------------------------------
// lattice layout
//
// Sites are stored parity-major (parity = sum of coordinates mod 2, even
// first).  Within a parity they are ordered block-major over "layout blocks"
// (power-of-two extents, the SAP blocks of the level), and inside a block by
// the lexicographic local index divided by two.  Block origins have even
// coordinates, so a site's parity equals the parity of its local coordinates.
// ---------------------------------------------------------------------------
struct Geom {
    int lex;      // 1: lexicographic layout (a coarsest lattice with an odd extent:
                  //    no parity structure); halves [0, vh) and [vh, 2 vh) of the
                  //    canonical order stand in for the two parities
    int d[4];     // lattice extents
    int b[4];     // layout block extents (powers of two, >= 2 for the fine level)
    int lb[4];    // log2 b
    int nb[4];    // blocks per dimension
    int bvh;      // sites per block and parity
    int lbvh;     // log2 bvh
    int vh;       // sites per parity
    int nblk;     // number of blocks
};

__host__ __device__ __forceinline__ int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) r++;
    return r;
}

__host__ __device__ __forceinline__ long canon_index(const int d[4], const int x[4]);
__host__ __device__ __forceinline__ void canon_coords(const int d[4], long i, int x[4]);

// coordinates of the site with parity p and layout index i
__host__ __device__ __forceinline__ void cb_coords(const Geom& g, int p, int i, int x[4]) {
    if (g.lex) {
        canon_coords(g.d, (long)p * g.vh + i, x);
        return;
    }
    int blk = i >> g.lbvh;
    int loc = i & (g.bvh - 1);
    int bc3 = blk % g.nb[3]; blk /= g.nb[3];
    int bc2 = blk % g.nb[2]; blk /= g.nb[2];
    int bc1 = blk % g.nb[1];
    int bc0 = blk / g.nb[1];
    int hb3 = g.b[3] >> 1;
    int l3h = loc & (hb3 - 1);
    int r = loc >> (g.lb[3] - 1);
    int l2 = r & (g.b[2] - 1); r >>= g.lb[2];
    int l1 = r & (g.b[1] - 1);
    int l0 = r >> g.lb[1];
    int q = (p + l0 + l1 + l2) & 1;
    x[0] = (bc0 << g.lb[0]) + l0;
    x[1] = (bc1 << g.lb[1]) + l1;
    x[2] = (bc2 << g.lb[2]) + l2;
    x[3] = (bc3 << g.lb[3]) + 2 * l3h + q;
}

// layout index of coordinates x (parity implied by the coordinates; in the
// lexicographic layout the index within the half that holds x)
__host__ __device__ __forceinline__ int cb_index(const Geom& g, const int x[4]) {
    if (g.lex) {
        const long c = canon_index(g.d, x);
        return (int)(c >= g.vh ? c - g.vh : c);
    }
    int blk = (((x[0] >> g.lb[0]) * g.nb[1] + (x[1] >> g.lb[1])) * g.nb[2] + (x[2] >> g.lb[2])) * g.nb[3] + (x[3] >> g.lb[3]);
    int loc = ((((x[0] & (g.b[0] - 1)) << g.lb[1] | (x[1] & (g.b[1] - 1))) << g.lb[2] | (x[2] & (g.b[2] - 1))) << g.lb[3] |
               (x[3] & (g.b[3] - 1))) >> 1;
    return (blk << g.lbvh) + loc;
}

__host__ __device__ __forceinline__ int site_parity(const int x[4]) { return (x[0] + x[1] + x[2] + x[3]) & 1; }

// the half of the layout that holds x: its parity, or in the lexicographic
// layout the half of the canonical order
__host__ __device__ __forceinline__ int lay_parity(const Geom& g, const int x[4]) {
    return g.lex ? (canon_index(g.d, x) >= g.vh ? 1 : 0) : site_parity(x);
}
// index of x in the whole layout (both halves)
__host__ __device__ __forceinline__ size_t lay_global(const Geom& g, const int x[4]) {
    return (size_t)lay_parity(g, x) * g.vh + cb_index(g, x);
}

__host__ __device__ __forceinline__ long canon_index(const int d[4], const int x[4]) {
    return (((long)x[0] * d[1] + x[1]) * d[2] + x[2]) * d[3] + x[3];
}

__host__ __device__ __forceinline__ void canon_coords(const int d[4], long i, int x[4]) {
    x[3] = (int)(i % d[3]); i /= d[3];
    x[2] = (int)(i % d[2]); i /= d[2];
    x[1] = (int)(i % d[1]);
    x[0] = (int)(i / d[1]);
}

// neighbour coordinates: k < 4 -> x + k, k >= 4 -> x - (k-4)
__host__ __device__ __forceinline__ void nb_coords(const Geom& g, const int x[4], int k, int y[4]) {
    y[0] = x[0]; y[1] = x[1]; y[2] = x[2]; y[3] = x[3];
    int mu = k & 3;
    if (k < 4) y[mu] = (x[mu] + 1 == g.d[mu]) ? 0 : x[mu] + 1;
    else y[mu] = (x[mu] == 0) ? g.d[mu] - 1 : x[mu] - 1;
}

// layout index of neighbour k of x, written with selects only (no dynamically
// indexed private arrays, so rolled loops stay in registers)
__device__ __forceinline__ int nb_index_sel(const Geom& g, const int x[4], int k) {
    const int mu = k & 3;
    const bool fwd = k < 4;
    int y[4];
#pragma unroll
    for (int nu = 0; nu < 4; nu++) {
        const int c = x[nu], d = g.d[nu];
        const int stepped = fwd ? ((c + 1 == d) ? 0 : c + 1) : ((c == 0) ? d - 1 : c - 1);
        y[nu] = (nu == mu) ? stepped : c;
    }
    return cb_index(g, y);
}

// whole-layout index of neighbour k of x, where x lies in half p (the other
// parity in the parity layout; looked up in the lexicographic one)
__device__ __forceinline__ size_t nb_global(const Geom& g, int p, const int x[4], int k) {
    if (g.lex) {
        int y[4];
        nb_coords(g, x, k, y);
        return (size_t)canon_index(g.d, y);
    }
    return (size_t)(1 - p) * g.vh + nb_index_sel(g, x, k);
}

// ---------------------------------------------------------------------------
// spin structure.  In the chiral representation every gamma_mu is
// [[0, B_mu], [B_mu^H, 0]] in the spin halves {0,1} / {2,3} with
//   B_0 = [[0, i], [i, 0]], B_1 = [[0, -1], [1, 0]], B_2 = [[i, 0], [0, -i]], B_3 = I.
// Hence (I -/+ gamma_mu) psi = (h, -/+ B_mu^H h) with h = psi_up -/+ B_mu psi_lo:
// a hop only needs the colour matrix applied to the two-spinor h.
// Spinor index: spin*3 + colour.
// ---------------------------------------------------------------------------
template <class T>
__host__ __device__ __forceinline__ void spin_project(int mu, T sgn, const cx<T> psi[12], cx<T> h[6]) {
    // h = psi_up + sgn * B_mu psi_lo
    for (int c = 0; c < 3; c++) {
        cx<T> lo0 = psi[6 + c], lo1 = psi[9 + c], b0, b1;
        switch (mu) {
            case 0: b0 = times_i(lo1); b1 = times_i(lo0); break;
            case 1: b0 = -lo1; b1 = lo0; break;
            case 2: b0 = times_i(lo0); b1 = times_mi(lo1); break;
            default: b0 = lo0; b1 = lo1; break;
        }
        h[c] = psi[c] + sgn * b0;
        h[3 + c] = psi[3 + c] + sgn * b1;
    }
}

template <class T>
__host__ __device__ __forceinline__ void spin_reconstruct(int mu, T sgn, const cx<T> g[6], cx<T> acc[12]) {
    // acc_up += g ; acc_lo += sgn * B_mu^H g
    for (int c = 0; c < 3; c++) {
        cx<T> w0 = g[c], w1 = g[3 + c], b0, b1;
        switch (mu) {
            case 0: b0 = times_mi(w1); b1 = times_mi(w0); break;
            case 1: b0 = w1; b1 = -w0; break;
            case 2: b0 = times_mi(w0); b1 = times_i(w1); break;
            default: b0 = w0; b1 = w1; break;
        }
        acc[c] += w0;
        acc[3 + c] += w1;
        acc[6 + c] += sgn * b0;
        acc[9 + c] += sgn * b1;
    }
}

// g = U h (dag = false) or U^H h (dag = true), per spin component of the two-spinor
template <class T>
__host__ __device__ __forceinline__ void su3_two_spinor(const cx<T> u[9], bool dag, const cx<T> h[6], cx<T> g[6]) {
    for (int s = 0; s < 2; s++)
        for (int a = 0; a < 3; a++) {
            cx<T> acc = dag ? cmulc(u[a], h[s * 3]) : u[a * 3] * h[s * 3];
            for (int b = 1; b < 3; b++) {
                if (dag) cmacc(acc, u[b * 3 + a], h[s * 3 + b]);
                else cmac(acc, u[a * 3 + b], h[s * 3 + b]);
            }
            g[s * 3 + a] = acc;
        }
}

// ---------------------------------------------------------------------------
// packed Hermitian 6x6 block: 6 real diagonal entries, then the 15 upper
// off-diagonal entries (i < j, row-major) as (re, im) pairs: 36 reals.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int herm_off(int i, int j) { return i * 6 - (i * (i + 1)) / 2 + (j - i - 1); }

template <class T>
__host__ __device__ __forceinline__ void herm6_apply(const T m[36], const cx<T>* in, cx<T>* out) {
#pragma unroll
    for (int i = 0; i < 6; i++) {
        cx<T> acc = m[i] * in[i];
#pragma unroll
        for (int j = 0; j < 6; j++) {
            if (j == i) continue;
            if (j > i) {
                int k = herm_off(i, j);
                cmac(acc, cx<T>{m[6 + 2 * k], m[7 + 2 * k]}, in[j]);
            } else {
                int k = herm_off(j, i);
                cmacc(acc, cx<T>{m[6 + 2 * k], m[7 + 2 * k]}, in[j]);
            }
        }
        out[i] = acc;
    }
}

// ---------------------------------------------------------------------------
// workgroup scheduling.  Consecutive workgroups of a grid are dealt round
// robin to the eight XCDs, each with its own L2.  xcd_swizzle maps the
// hardware index w to a logical one so that XCD x works on the contiguous
// range [x n/8, (x+1) n/8) of logical workgroups, which keeps lattice
// neighbours (halo reuse) in one L2.  Grids whose size is not a multiple of 8
// keep the identity.
// ---------------------------------------------------------------------------
static constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_swizzle(int w, int n) {
    if (n % NUM_XCD) return w;
    return (w % NUM_XCD) * (n / NUM_XCD) + w / NUM_XCD;
}

// ---------------------------------------------------------------------------
// reductions (wave64 shuffles, then one LDS step across the waves)
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over the workgroup, returned to every thread.  `scratch` must hold
// at least blockDim.x/64 values; the call synchronises the workgroup twice.
template <class T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
    v = wave_sum(v);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < nw; i++) s += scratch[i];
    return s;
}

}  // namespace dd
