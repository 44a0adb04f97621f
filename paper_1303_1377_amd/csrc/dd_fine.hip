// dd_fine.hip -- fine-level kernels of DD-alpha-AMG on gfx950.
//
//   clover-Wilson stencil ............ explicit site form of D (Sec. 2.2)
//   clover term ...................... eq. (lattice_WD), four-leaf Q_{mu nu}
//   SAP half sweep ................... Sec. 2.3 with the odd-even MR block solver of Sec. 5
//   restriction / prolongation ....... eq. (aggInterpolation), standard aggregation (Sec. 3.2)
//   local Gram-Schmidt ............... Sec. 3.1 (local orthonormalisation of the test vectors)
//   coarse-operator assembly ......... D_c = P^H D P as a nearest-neighbour stencil (Sec. 3.2)
//
// Data layout: even-odd, block-major, structure of arrays (see dd_common.h).
// A spinor field is [parity][12][vh] complex, the links [parity][mu][9][vh],
// packed clover blocks [parity][72][vh] reals.  One thread owns one site, so
// every load of a component is coalesced across the wavefront.
#include <mutex>

#include "dd_kernels.h"

#include <math.h>

namespace dd {

static inline int nblk_of(long n, int b) { return (int)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// layout conversion
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_import_gauge(Geom g, const double* __restrict__ canon, cx<T>* __restrict__ U) {
    long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long vol = 2L * g.vh;
    if (s >= vol) return;
    int x[4];
    canon_coords(g.d, s, x);
    int p = site_parity(x), i = cb_index(g, x);
    const cx<double>* src = reinterpret_cast<const cx<double>*>(canon) + s * 36;
    for (int mu = 0; mu < 4; mu++)
        for (int e = 0; e < 9; e++) U[((size_t)(p * 4 + mu) * 9 + e) * g.vh + i] = ccast<T>(src[mu * 9 + e]);
}

template <class T>
__global__ void k_import_vectors(Geom g, int n, const double* __restrict__ canon, cx<T>* __restrict__ out) {
    long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long vol = 2L * g.vh;
    if (s >= vol) return;
    int x[4];
    canon_coords(g.d, s, x);
    int p = site_parity(x), i = cb_index(g, x);
    const cx<double>* src = reinterpret_cast<const cx<double>*>(canon);
    for (int v = 0; v < n; v++)
        for (int c = 0; c < 12; c++)
            out[(size_t)v * 24 * g.vh + (size_t)(p * 12 + c) * g.vh + i] = ccast<T>(src[((size_t)v * vol + s) * 12 + c]);
}

template <class T>
__global__ void k_export_vectors(Geom g, int n, const cx<T>* __restrict__ in, double* __restrict__ canon) {
    long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long vol = 2L * g.vh;
    if (s >= vol) return;
    int x[4];
    canon_coords(g.d, s, x);
    int p = site_parity(x), i = cb_index(g, x);
    cx<double>* dst = reinterpret_cast<cx<double>*>(canon);
    for (int v = 0; v < n; v++)
        for (int c = 0; c < 12; c++)
            dst[((size_t)v * vol + s) * 12 + c] = ccast<double>(in[(size_t)v * 24 * g.vh + (size_t)(p * 12 + c) * g.vh + i]);
}

template <class T>
void fine_import_gauge(const Geom& g, const double* canon, cx<T>* U, hipStream_t s) {
    long vol = 2L * g.vh;
    k_import_gauge<T><<<nblk_of(vol, 256), 256, 0, s>>>(g, canon, U);
}
template <class T>
void fine_import_spinor(const Geom& g, const double* canon, cx<T>* out, hipStream_t s) {
    long vol = 2L * g.vh;
    k_import_vectors<T><<<nblk_of(vol, 256), 256, 0, s>>>(g, 1, canon, out);
}
template <class T>
void fine_export_spinor(const Geom& g, const cx<T>* in, double* canon, hipStream_t s) {
    long vol = 2L * g.vh;
    k_export_vectors<T><<<nblk_of(vol, 256), 256, 0, s>>>(g, 1, in, canon);
}
template <class T>
void fine_import_vectors(const Geom& g, int n, const double* canon, cx<T>* out, hipStream_t s) {
    long vol = 2L * g.vh;
    k_import_vectors<T><<<nblk_of(vol, 256), 256, 0, s>>>(g, n, canon, out);
}
template <class T>
void fine_export_vectors(const Geom& g, int n, const cx<T>* in, double* canon, hipStream_t s) {
    long vol = 2L * g.vh;
    k_export_vectors<T><<<nblk_of(vol, 256), 256, 0, s>>>(g, n, in, canon);
}

// ---------------------------------------------------------------------------
// clover term
// ---------------------------------------------------------------------------
__device__ __forceinline__ cx<double> Bmat(int mu, int r, int c) {
    // the off-diagonal spin blocks of the chiral gamma matrices (dd_common.h)
    switch (mu) {
        case 0: return (r != c) ? cx<double>{0.0, 1.0} : cx<double>{0.0, 0.0};
        case 1: return (r == 0 && c == 1) ? cx<double>{-1.0, 0.0} : (r == 1 && c == 0) ? cx<double>{1.0, 0.0} : cx<double>{0.0, 0.0};
        case 2: return (r != c) ? cx<double>{0.0, 0.0} : (r == 0 ? cx<double>{0.0, 1.0} : cx<double>{0.0, -1.0});
        default: return (r == c) ? cx<double>{1.0, 0.0} : cx<double>{0.0, 0.0};
    }
}

__device__ __forceinline__ void load_link64(const Geom& g, const cx<double>* U, const int y[4], int mu, cx<double> u[9]) {
    int p = site_parity(y), i = cb_index(g, y);
    for (int e = 0; e < 9; e++) u[e] = U[((size_t)(p * 4 + mu) * 9 + e) * g.vh + i];
}

__device__ __forceinline__ void m3mul(const cx<double> a[9], const cx<double> b[9], cx<double> c[9]) {
    cx<double> t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cx<double> s = czero<double>();
            for (int k = 0; k < 3; k++) s += a[i * 3 + k] * b[k * 3 + j];
            t[i * 3 + j] = s;
        }
    for (int e = 0; e < 9; e++) c[e] = t[e];
}
// c = a b^H
__device__ __forceinline__ void m3mul_nh(const cx<double> a[9], const cx<double> b[9], cx<double> c[9]) {
    cx<double> t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cx<double> s = czero<double>();
            for (int k = 0; k < 3; k++) s += a[i * 3 + k] * conj(b[j * 3 + k]);
            t[i * 3 + j] = s;
        }
    for (int e = 0; e < 9; e++) c[e] = t[e];
}
// c = a^H b
__device__ __forceinline__ void m3mul_hn(const cx<double> a[9], const cx<double> b[9], cx<double> c[9]) {
    cx<double> t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cx<double> s = czero<double>();
            for (int k = 0; k < 3; k++) s += cmulc(a[k * 3 + i], b[k * 3 + j]);
            t[i * 3 + j] = s;
        }
    for (int e = 0; e < 9; e++) c[e] = t[e];
}

// Gauss-Jordan inverse of a 6x6 complex matrix (partial pivoting); returns 0 if singular
__device__ int inv6(cx<double> a[36], cx<double> r[36]) {
    for (int i = 0; i < 36; i++) r[i] = czero<double>();
    for (int i = 0; i < 6; i++) r[i * 7] = cx<double>{1.0, 0.0};
    for (int c = 0; c < 6; c++) {
        int p = c;
        double best = norm2(a[c * 6 + c]);
        for (int q = c + 1; q < 6; q++)
            if (norm2(a[q * 6 + c]) > best) { best = norm2(a[q * 6 + c]); p = q; }
        if (best == 0.0) return 0;
        if (p != c)
            for (int j = 0; j < 6; j++) {
                cx<double> t = a[c * 6 + j]; a[c * 6 + j] = a[p * 6 + j]; a[p * 6 + j] = t;
                t = r[c * 6 + j]; r[c * 6 + j] = r[p * 6 + j]; r[p * 6 + j] = t;
            }
        cx<double> piv = a[c * 6 + c];
        double d = norm2(piv);
        cx<double> ip = {piv.re / d, -piv.im / d};
        for (int j = 0; j < 6; j++) { a[c * 6 + j] = a[c * 6 + j] * ip; r[c * 6 + j] = r[c * 6 + j] * ip; }
        for (int q = 0; q < 6; q++) {
            if (q == c) continue;
            cx<double> f = a[q * 6 + c];
            for (int j = 0; j < 6; j++) {
                a[q * 6 + j] -= f * a[c * 6 + j];
                r[q * 6 + j] -= f * r[c * 6 + j];
            }
        }
    }
    return 1;
}

__device__ __forceinline__ void pack_herm(const cx<double> m[36], double* dst, int vh, int i) {
    for (int r = 0; r < 6; r++) dst[(size_t)r * vh + i] = m[r * 7].re;
    for (int r = 0; r < 6; r++)
        for (int c = r + 1; c < 6; c++) {
            int k = herm_off(r, c);
            dst[(size_t)(6 + 2 * k) * vh + i] = m[r * 6 + c].re;
            dst[(size_t)(7 + 2 * k) * vh + i] = m[r * 6 + c].im;
        }
}

__device__ __forceinline__ void unpack_herm(const double* src, int vh, int i, cx<double> m[36]) {
    for (int r = 0; r < 6; r++) m[r * 7] = cx<double>{src[(size_t)r * vh + i], 0.0};
    for (int r = 0; r < 6; r++)
        for (int c = r + 1; c < 6; c++) {
            int k = herm_off(r, c);
            cx<double> v = {src[(size_t)(6 + 2 * k) * vh + i], src[(size_t)(7 + 2 * k) * vh + i]};
            m[r * 6 + c] = v;
            m[c * 6 + r] = conj(v);
        }
}

// finish one chiral block: pack A and its inverse
__device__ __forceinline__ void finish_block(cx<double> a[36], double* clov, double* clovinv, int p, int h, int vh, int i,
                                             int* bad) {
    pack_herm(a, clov + (size_t)(p * 72 + h * 36) * vh, vh, i);
    cx<double> r[36];
    if (!inv6(a, r)) atomicAdd(bad, 1);
    pack_herm(r, clovinv + (size_t)(p * 72 + h * 36) * vh, vh, i);
}

// T(x) = -(csw/32) sum_{mu,nu} gamma_mu gamma_nu (x) (Q_{mu nu} - Q_{nu mu})
//      = -(csw/16) sum_{mu<nu} diag(B_mu B_nu^H, B_mu^H B_nu) (x) (Q_{mu nu} - Q_{mu nu}^H)
__global__ void k_clover_links(Geom g, const cx<double>* __restrict__ U, double m0, double csw, double* clov,
                               double* clovinv, int* bad) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 2 * g.vh) return;
    int p = gid >= g.vh, i = gid - p * g.vh;
    int x[4];
    cb_coords(g, p, i, x);
    cx<double> Tb[2][36];
    for (int h = 0; h < 2; h++)
        for (int e = 0; e < 36; e++) Tb[h][e] = czero<double>();
    for (int mu = 0; mu < 4; mu++)
        for (int nu = mu + 1; nu < 4; nu++) {
            int xpm[4], xpn[4], xmm[4], xmn[4], xmmpn[4], xmmmn[4], xmnpm[4];
            nb_coords(g, x, mu, xpm);
            nb_coords(g, x, nu, xpn);
            nb_coords(g, x, 4 + mu, xmm);
            nb_coords(g, x, 4 + nu, xmn);
            nb_coords(g, xmm, nu, xmmpn);
            nb_coords(g, xmm, 4 + nu, xmmmn);
            nb_coords(g, xmn, mu, xmnpm);
            cx<double> q[9], t[9], a[9], b[9];
            // U_mu(x) U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H
            load_link64(g, U, x, mu, a); load_link64(g, U, xpm, nu, b); m3mul(a, b, t);
            load_link64(g, U, xpn, mu, a); m3mul_nh(t, a, t);
            load_link64(g, U, x, nu, a); m3mul_nh(t, a, q);
            // U_nu(x) U_mu(x-mu+nu)^H U_nu(x-mu)^H U_mu(x-mu)
            load_link64(g, U, x, nu, a); load_link64(g, U, xmmpn, mu, b); m3mul_nh(a, b, t);
            load_link64(g, U, xmm, nu, a); m3mul_nh(t, a, t);
            load_link64(g, U, xmm, mu, a); m3mul(t, a, t);
            for (int e = 0; e < 9; e++) q[e] += t[e];
            // U_mu(x-mu)^H U_nu(x-mu-nu)^H U_mu(x-mu-nu) U_nu(x-nu)
            load_link64(g, U, xmm, mu, a); load_link64(g, U, xmmmn, nu, b);
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) {  // t = a^H b^H = (b a)^H
                    cx<double> s = czero<double>();
                    for (int k = 0; k < 3; k++) s += b[r * 3 + k] * a[k * 3 + c];
                    t[c * 3 + r] = conj(s);
                }
            load_link64(g, U, xmmmn, mu, a); m3mul(t, a, t);
            load_link64(g, U, xmn, nu, a); m3mul(t, a, t);
            for (int e = 0; e < 9; e++) q[e] += t[e];
            // U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^H
            load_link64(g, U, xmn, nu, a); load_link64(g, U, xmn, mu, b); m3mul_hn(a, b, t);
            load_link64(g, U, xmnpm, nu, a); m3mul(t, a, t);
            load_link64(g, U, x, mu, a); m3mul_nh(t, a, t);
            for (int e = 0; e < 9; e++) q[e] += t[e];
            // F = Q - Q^H
            cx<double> F[9];
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) F[r * 3 + c] = q[r * 3 + c] - conj(q[c * 3 + r]);
            for (int h = 0; h < 2; h++) {
                // sigma = B_mu B_nu^H (h = 0) or B_mu^H B_nu (h = 1)
                cx<double> sg[4];
                for (int r = 0; r < 2; r++)
                    for (int c = 0; c < 2; c++) {
                        cx<double> s = czero<double>();
                        for (int k = 0; k < 2; k++) {
                            if (h == 0) s += Bmat(mu, r, k) * conj(Bmat(nu, c, k));
                            else s += conj(Bmat(mu, k, r)) * Bmat(nu, k, c);
                        }
                        sg[r * 2 + c] = s;
                    }
                for (int sr = 0; sr < 2; sr++)
                    for (int sc = 0; sc < 2; sc++)
                        for (int a3 = 0; a3 < 3; a3++)
                            for (int b3 = 0; b3 < 3; b3++)
                                Tb[h][(sr * 3 + a3) * 6 + sc * 3 + b3] += (-csw / 16.0) * (sg[sr * 2 + sc] * F[a3 * 3 + b3]);
            }
        }
    for (int h = 0; h < 2; h++) {
        for (int e = 0; e < 6; e++) Tb[h][e * 7].re += m0 + 4.0;
        finish_block(Tb[h], clov, clovinv, p, h, g.vh, i, bad);
    }
}

// user-supplied T(x): canonical [vol][2][6][6] complex
__global__ void k_clover_user(Geom g, const double* __restrict__ canonT, double m0, double* clov, double* clovinv,
                              int* bad) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 2 * g.vh) return;
    int p = gid >= g.vh, i = gid - p * g.vh;
    int x[4];
    cb_coords(g, p, i, x);
    long s = canon_index(g.d, x);
    const cx<double>* src = reinterpret_cast<const cx<double>*>(canonT) + s * 72;
    for (int h = 0; h < 2; h++) {
        cx<double> a[36];
        for (int e = 0; e < 36; e++) a[e] = src[h * 36 + e];
        for (int e = 0; e < 6; e++) a[e * 7].re += m0 + 4.0;
        finish_block(a, clov, clovinv, p, h, g.vh, i, bad);
    }
}

__global__ void k_clover_shift(Geom g, double dm, double* clov, double* clovinv, int* bad) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 2 * g.vh) return;
    int p = gid >= g.vh, i = gid - p * g.vh;
    for (int h = 0; h < 2; h++) {
        cx<double> a[36];
        unpack_herm(clov + (size_t)(p * 72 + h * 36) * g.vh, g.vh, i, a);
        for (int e = 0; e < 6; e++) a[e * 7].re += dm;
        finish_block(a, clov, clovinv, p, h, g.vh, i, bad);
    }
}

__global__ void k_clover_export(Geom g, const double* __restrict__ packed, double* __restrict__ canon) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 2 * g.vh) return;
    int p = gid >= g.vh, i = gid - p * g.vh;
    int x[4];
    cb_coords(g, p, i, x);
    long s = canon_index(g.d, x);
    cx<double>* dst = reinterpret_cast<cx<double>*>(canon) + s * 72;
    for (int h = 0; h < 2; h++) {
        cx<double> a[36];
        unpack_herm(packed + (size_t)(p * 72 + h * 36) * g.vh, g.vh, i, a);
        for (int e = 0; e < 36; e++) dst[h * 36 + e] = a[e];
    }
}

void fine_clover_from_links(const Geom& g, const cx<double>* U, double m0, double csw, double* clov, double* clovinv,
                            int* bad, hipStream_t s) {
    k_clover_links<<<nblk_of(2L * g.vh, 128), 128, 0, s>>>(g, U, m0, csw, clov, clovinv, bad);
}
void fine_clover_from_user(const Geom& g, const double* canonT, double m0, double* clov, double* clovinv, int* bad,
                           hipStream_t s) {
    k_clover_user<<<nblk_of(2L * g.vh, 128), 128, 0, s>>>(g, canonT, m0, clov, clovinv, bad);
}
void fine_clover_shift(const Geom& g, double dm, double* clov, double* clovinv, int* bad, hipStream_t s) {
    k_clover_shift<<<nblk_of(2L * g.vh, 128), 128, 0, s>>>(g, dm, clov, clovinv, bad);
}
void fine_clover_export(const Geom& g, const double* packed, double* canon, hipStream_t s) {
    k_clover_export<<<nblk_of(2L * g.vh, 256), 256, 0, s>>>(g, packed, canon);
}

// ---------------------------------------------------------------------------
// stencil building blocks
// ---------------------------------------------------------------------------
template <class T, class S>
__device__ __forceinline__ void load_link(const FineOp<T, S>& op, int p, int mu, int i, cx<T> u[9]) {
    const cx<S>* base = op.U + (size_t)(p * 4 + mu) * 9 * op.g.vh + i;
#pragma unroll
    for (int e = 0; e < 9; e++) u[e] = ccast<T>(base[(size_t)e * op.g.vh]);
}

template <class T, class S>
__device__ __forceinline__ void load_spinor(const cx<S>* psi, int vh, int p, int i, cx<T> v[12]) {
    const cx<S>* base = psi + (size_t)p * 12 * vh + i;
#pragma unroll
    for (int c = 0; c < 12; c++) v[c] = ccast<T>(base[(size_t)c * vh]);
}

template <class T>
__device__ __forceinline__ void store_spinor(cx<T>* psi, int vh, int p, int i, const cx<T> v[12]) {
    cx<T>* base = psi + (size_t)p * 12 * vh + i;
#pragma unroll
    for (int c = 0; c < 12; c++) base[(size_t)c * vh] = v[c];
}

// chirality half h of the site (p, i) of an FP16 spinor set (see hspin)
template <class T>
__device__ __forceinline__ void half_load(const hspin& psi, int vh, int p, int h, int i, cx<T> v[6]) {
    const hpair* base = psi.d + (size_t)((2 * p + h) * 7) * vh + i;
    const float sc = __builtin_bit_cast(float, base[(size_t)6 * vh]);
#pragma unroll
    for (int c = 0; c < 6; c++) {
        const hpair q = base[(size_t)c * vh];
        v[c] = {T((float)q.x * sc), T((float)q.y * sc)};
    }
}
template <class T>
__device__ __forceinline__ void half_store(const hspin& psi, int vh, int p, int h, int i, const cx<T> v[6]) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 6; c++) m = fmaxf(m, fmaxf(fabsf((float)v[c].re), fabsf((float)v[c].im)));
    const float inv = m > 0.f ? 1.f / m : 0.f;
    hpair* base = psi.d + (size_t)((2 * p + h) * 7) * vh + i;
#pragma unroll
    for (int c = 0; c < 6; c++) {
        hpair q;
        q.x = (_Float16)((float)v[c].re * inv);
        q.y = (_Float16)((float)v[c].im * inv);
        base[(size_t)c * vh] = q;
    }
    base[(size_t)6 * vh] = __builtin_bit_cast(hpair, m);
}
template <class T>
__device__ __forceinline__ void load_spinor(const hspin& psi, int vh, int p, int i, cx<T> v[12]) {
    half_load(psi, vh, p, 0, i, v);
    half_load(psi, vh, p, 1, i, v + 6);
}
template <class T>
__device__ __forceinline__ void store_spinor(const hspin& psi, int vh, int p, int i, const cx<T> v[12]) {
    half_store(psi, vh, p, 0, i, v);
    half_store(psi, vh, p, 1, i, v + 6);
}
// a vector pointer with __restrict__ for plain spinor sets (FP16 sets are a struct)
template <class VP> struct vrestrict { using type = VP; };
template <class T> struct vrestrict<cx<T>*> { using type = cx<T>* __restrict__; };

// out = A v with the packed clover blocks at (p, i) of array `cl`
template <class T, class S>
__device__ __forceinline__ void clover_apply(const S* __restrict__ cl, int vh, int p, int i, const cx<T> v[12], cx<T> out[12]) {
#pragma unroll
    for (int h = 0; h < 2; h++) {
        T m[36];
        const S* base = cl + (size_t)(p * 72 + h * 36) * vh + i;
#pragma unroll
        for (int r = 0; r < 36; r++) m[r] = T(base[(size_t)r * vh]);
        herm6_apply(m, v + 6 * h, out + 6 * h);
    }
}

// acc += (I -/+ gamma_mu) (x) U psi_y for hop k from a site of parity p:
// forward (k < 4): link U_mu(x) at (p, i); backward: U_mu(y)^H at (1-p, j)
template <class T, class S>
__device__ __forceinline__ void hop_accum(const FineOp<T, S>& op, int k, int p, int i, int j, const cx<T> v[12], cx<T> acc[12]) {
    int mu = k & 3;
    cx<T> h[6], gg[6], u[9];
    if (k < 4) {
        spin_project(mu, T(-1), v, h);
        load_link(op, p, mu, i, u);
        su3_two_spinor(u, false, h, gg);
        spin_reconstruct(mu, T(-1), gg, acc);
    } else {
        spin_project(mu, T(1), v, h);
        load_link(op, 1 - p, mu, j, u);
        su3_two_spinor(u, true, h, gg);
        spin_reconstruct(mu, T(1), gg, acc);
    }
}

// ---------------------------------------------------------------------------
// D psi = A psi - 1/2 sum_mu [(I - g_mu) U_mu(x) psi(x+mu) + (I + g_mu) U_mu(x-mu)^H psi(x-mu)]
// one thread per site, both parities in one grid.  With SCHED_FUSED a
// workgroup takes the even and the odd sites of the same layout blocks, so the
// forward links its even sites read are the backward links of its odd sites
// (and the spinors one parity gathers were loaded by the other): every link
// and spinor is fetched from HBM about once.  Without it the grid runs all
// even sites, then all odd ones, and each link is fetched twice.
// ---------------------------------------------------------------------------
template <class T, class S, class TI = T>
__global__ void __launch_bounds__(256) k_dirac(FineOp<T, S> op, const cx<TI>* __restrict__ in, cx<T>* __restrict__ out,
                                               long ld, Mask mk) {
    const Geom g = op.g;
    const int w = (op.sched & SCHED_XCD) ? xcd_swizzle(blockIdx.x, gridDim.x) : blockIdx.x;
    const int gid = w * blockDim.x + threadIdx.x;
    if (gid >= 2 * g.vh || !mk.on(blockIdx.y)) return;
    in += blockIdx.y * ld;
    out += blockIdx.y * ld;
    int p, i;
    if (op.sched & (SCHED_FUSED | SCHED_LDS)) {
        p = (gid >> g.lbvh) & 1;
        i = ((gid >> (g.lbvh + 1)) << g.lbvh) | (gid & (g.bvh - 1));
    } else {
        p = gid >= g.vh;
        i = gid - p * g.vh;
    }
    int x[4];
    cb_coords(g, p, i, x);
    cx<T> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = czero<T>();
    // hops in the order +0, -0, +1, -1, ... (the order of the LDS schedule, so
    // that every schedule produces the same bits)
#pragma unroll
    for (int kk = 0; kk < 8; kk++) {
        const int k = (kk >> 1) + ((kk & 1) << 2);
        int y[4];
        nb_coords(g, x, k, y);
        int j = cb_index(g, y);
        cx<T> v[12];
        load_spinor(in, g.vh, 1 - p, j, v);
        hop_accum(op, k, p, i, j, v, acc);
    }
    cx<T> v[12], a[12];
    load_spinor(in, g.vh, p, i, v);
    clover_apply(op.clov, g.vh, p, i, v, a);
#pragma unroll
    for (int c = 0; c < 12; c++) a[c] -= T(0.5) * acc[c];
    store_spinor(out, g.vh, p, i, a);
}

// ---------------------------------------------------------------------------
// One parity of the odd-even reduced operator (the odd-even preconditioned
// BiCGStab of the comparison solver, Sec. 6): with p the parity written,
// q = 1 - p, D_pq = -1/2 H_pq the hopping between the parities and A_pp the
// clover blocks,
//   out_p = M ( s * P self_p + c * D_pq in_q ),
// P = A_pp when PRE_A else I, M = A_pp^{-1} when POST_INV else I.  The hops
// run in the order of the full stencil.  One thread per site of parity p.
// ---------------------------------------------------------------------------
template <class T, class S, bool PRE_A, bool POST_INV>
__global__ void __launch_bounds__(256) k_oe_hop(FineOp<T, S> op, int p, const cx<T>* __restrict__ self,
                                                const cx<T>* __restrict__ in, cx<T>* __restrict__ out, T sc, T cc) {
    const Geom g = op.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.vh) return;
    int x[4];
    cb_coords(g, p, i, x);
    cx<T> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = czero<T>();
    if (cc != T(0)) {
#pragma unroll
        for (int kk = 0; kk < 8; kk++) {
            const int k = (kk >> 1) + ((kk & 1) << 2);
            int y[4];
            nb_coords(g, x, k, y);
            const int j = cb_index(g, y);
            cx<T> v[12];
            load_spinor(in, g.vh, 1 - p, j, v);
            hop_accum(op, k, p, i, j, v, acc);
        }
    }
    cx<T> a[12];
    if (sc != T(0)) {
        cx<T> v[12];
        load_spinor(self, g.vh, p, i, v);
        if (PRE_A) clover_apply(op.clov, g.vh, p, i, v, a);
        else
#pragma unroll
            for (int c = 0; c < 12; c++) a[c] = v[c];
#pragma unroll
        for (int c = 0; c < 12; c++) a[c] = sc * a[c];
    } else {
#pragma unroll
        for (int c = 0; c < 12; c++) a[c] = czero<T>();
    }
    const T hc = T(-0.5) * cc;
#pragma unroll
    for (int c = 0; c < 12; c++) a[c] += hc * acc[c];
    if (POST_INV) {
        cx<T> b[12];
        clover_apply(op.clovinv, g.vh, p, i, a, b);
        store_spinor(out, g.vh, p, i, b);
    } else {
        store_spinor(out, g.vh, p, i, a);
    }
}

template <class T, class S>
void fine_oe_hop(const FineOp<T, S>& op, int p, bool pre_a, bool post_inv, double sc, double cc, const cx<T>* self,
                 const cx<T>* in, cx<T>* out, hipStream_t s) {
    const int nb = nblk_of(op.g.vh, 256);
    const T a = T(sc), b = T(cc);
    if (pre_a && post_inv) k_oe_hop<T, S, true, true><<<nb, 256, 0, s>>>(op, p, self, in, out, a, b);
    else if (pre_a) k_oe_hop<T, S, true, false><<<nb, 256, 0, s>>>(op, p, self, in, out, a, b);
    else if (post_inv) k_oe_hop<T, S, false, true><<<nb, 256, 0, s>>>(op, p, self, in, out, a, b);
    else k_oe_hop<T, S, false, false><<<nb, 256, 0, s>>>(op, p, self, in, out, a, b);
}

// ---------------------------------------------------------------------------
// Stencil with the layout block staged in LDS (SCHED_LDS).  One workgroup per
// layout block, one thread per site (threads [0, bvh) even, [bvh, 2 bvh) odd).
//   1. every thread copies its spinor into SP (coalesced; each spinor is read
//      from memory once by its own block);
//   2. per direction mu, with U = U_mu(x) loaded once by the owner x:
//      forward hop  acc(x)    += (I - g_mu) U psi(x+mu)      psi from SP if x+mu is in the block
//      backward hop acc(x+mu) += (I + g_mu) U^H psi(x)       computed by x, handed to
//                                                            x+mu through HB as the colour-
//                                                            rotated two-spinor
//      so each internal link is loaded once and applied twice; hops that
//      leave the block gather the link and spinor of the neighbour block;
//   3. out = A psi - acc / 2.
// LDS: SP [2][12][bvh] + HB [2][6][bvh] complex entries.
// ---------------------------------------------------------------------------
template <class T, class S, class TI = T>
__global__ void __launch_bounds__(256) k_dirac_lds(FineOp<T, S> op, const cx<TI>* __restrict__ in, cx<T>* __restrict__ out,
                                                   long ld, Mask mk, int nr) {
    extern __shared__ char smem_raw[];
    // one workgroup per (layout block, RHS), RHS fastest in the logical order:
    // the nr workgroups of a block run back to back on one XCD and the later
    // ones find the block's links and clover in its L2
    const int lw = (op.sched & SCHED_XCD) ? xcd_swizzle(blockIdx.x, gridDim.x) : blockIdx.x;
    const int rhs = lw % nr;
    if (!mk.on(rhs)) return;
    const Geom g = op.g;
    const int bvh = g.bvh;
    cx<T>* SP = reinterpret_cast<cx<T>*>(smem_raw);  // [2][12][bvh]
    cx<T>* HB = SP + 24 * bvh;                         // [2][6][bvh]
    in += rhs * ld;
    out += rhs * ld;
    const int blk = lw / nr;
    const int t = threadIdx.x;
    const int p = t >= bvh;
    const int l = t - p * bvh;
    const int base = blk << g.lbvh;
    const int i = base + l;
    {
        cx<T> v[12];
        load_spinor(in, g.vh, p, i, v);
#pragma unroll
        for (int c = 0; c < 12; c++) SP[(p * 12 + c) * bvh + l] = v[c];
    }
    int x[4];
    cb_coords(g, p, i, x);
    cx<T> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = czero<T>();
    __syncthreads();
    const int q = 1 - p;
#pragma unroll 1
    for (int mu = 0; mu < 4; mu++) {
        const int jf = nb_index_sel(g, x, mu);
        const int jb = nb_index_sel(g, x, 4 + mu);
        const bool inf = (jf >> g.lbvh) == blk, inb = (jb >> g.lbvh) == blk;
        cx<T> u[9], h[6], gg[6];
        load_link(op, p, mu, i, u);
        {
            // forward hop of x
            cx<T> v[12];
            if (inf) {
                const int lf = jf & (bvh - 1);
#pragma unroll
                for (int c = 0; c < 12; c++) v[c] = SP[(q * 12 + c) * bvh + lf];
            } else {
                load_spinor(in, g.vh, q, jf, v);
            }
            spin_project(mu, T(-1), v, h);
            su3_two_spinor(u, false, h, gg);
            spin_reconstruct(mu, T(-1), gg, acc);
        }
        if (inf) {
            // backward hop of x+mu, with the link just loaded
            cx<T> v[12];
#pragma unroll
            for (int c = 0; c < 12; c++) v[c] = SP[(p * 12 + c) * bvh + l];
            spin_project(mu, T(1), v, h);
            su3_two_spinor(u, true, h, gg);
            const int lf = jf & (bvh - 1);
#pragma unroll
            for (int c = 0; c < 6; c++) HB[(q * 6 + c) * bvh + lf] = gg[c];
        }
        __syncthreads();
        if (inb) {
#pragma unroll
            for (int c = 0; c < 6; c++) gg[c] = HB[(p * 6 + c) * bvh + l];
        } else {
            cx<T> v[12];
            load_spinor(in, g.vh, q, jb, v);
            load_link(op, q, mu, jb, u);
            spin_project(mu, T(1), v, h);
            su3_two_spinor(u, true, h, gg);
        }
        spin_reconstruct(mu, T(1), gg, acc);
        __syncthreads();
    }
    cx<T> v[12], a[12];
#pragma unroll
    for (int c = 0; c < 12; c++) v[c] = SP[(p * 12 + c) * bvh + l];
    clover_apply(op.clov, g.vh, p, i, v, a);
#pragma unroll
    for (int c = 0; c < 12; c++) a[c] -= T(0.5) * acc[c];
    store_spinor(out, g.vh, p, i, a);
}

template <class T>
size_t fine_dirac_lds_bytes(const Geom& g) {
    return sizeof(cx<T>) * 36 * (size_t)g.bvh;
}

// the LDS stencil needs whole waves and at most 256 threads per layout block
static inline bool dirac_lds_fits(const Geom& g) { return 2 * g.bvh >= 64 && 2 * g.bvh <= 256; }

template <class T, class S, class TI>
static void dirac_launch(const FineOp<T, S>& op, const cx<TI>* in, cx<T>* out, hipStream_t s, int nr, long ld, Mask mk) {
    if ((op.sched & SCHED_LDS) && dirac_lds_fits(op.g)) {
        const size_t lds = fine_dirac_lds_bytes<T>(op.g);
        static std::mutex mu;
        static size_t configured = 65536;
        static bool refused = false;
        size_t allowed;
        {
            std::lock_guard<std::mutex> lock(mu);
            if (lds > configured && !refused) {
                if (hipFuncSetAttribute((const void*)k_dirac_lds<T, S, TI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds) == hipSuccess)
                    configured = lds;
                else {
                    (void)hipGetLastError();
                    refused = true;
                }
            }
            allowed = configured;
        }
        if (lds <= allowed) {
            k_dirac_lds<T, S, TI><<<op.g.nblk * nr, 2 * op.g.bvh, lds, s>>>(op, in, out, ld, mk, nr);
            return;
        }
    }
    dim3 grid(nblk_of(2L * op.g.vh, 256), nr);
    k_dirac<T, S, TI><<<grid, 256, 0, s>>>(op, in, out, ld, mk);
}

template <class T, class S>
void fine_dirac(const FineOp<T, S>& op, const cx<T>* in, cx<T>* out, hipStream_t s, int nr, long ld, Mask mk) {
    dirac_launch<T, S, T>(op, in, out, s, nr, ld, mk);
}

void fine_dirac_from32(const FineOp<double>& op, const cx<float>* in, cx<double>* out, hipStream_t s, int nr, long ld,
                       Mask mk) {
    dirac_launch<double, double, float>(op, in, out, s, nr, ld, mk);
}

// ---------------------------------------------------------------------------
// SAP half sweep: one workgroup per lattice block of the active colour, two
// lanes per pair of block sites (the even and the odd site of one local layout
// index), each lane holding one chirality half of both.  With r = b - D z
// restricted to the block and H the hopping part of D:
//   t0_e = A_e^{-1}(b_e - (H z)_e) - z_e               (= A_ee^{-1} r_e)
//   f_o  = b_o - A_o z_o - (H z)_o - (H_int t0)_o        (= r_o - D_oe A_ee^{-1} r_e)
//   MR on S = A_oo - D_oe A_ee^{-1} D_eo (block-internal hops) from e_o = 0
//   e_e  = t0_e - A_e^{-1} (H_int e_o)_e
//   z   += e on the block
// The block's operator stays on chip for the whole half sweep: the links
// joining two sites of the block live in LDS as their first two rows (the
// third row of an SU(3) matrix is conj(row0 x row1)), each lane keeps its
// chirality half of the clover blocks (A^{-1} at the even, A at the odd site)
// in registers, and the block fields E (even) and O (odd) are exchanged
// through LDS.  Every
// link, clover entry and spinor is therefore read from memory once per half
// sweep.  The MR inner products are wavefront shuffles plus one LDS step.
// ---------------------------------------------------------------------------
struct LinkMap {        // compact index of the block-internal links of direction mu
    int ext[4][4];      // box extents per direction
    int off[4];         // offset of direction mu
    int total;
};

__host__ __device__ __forceinline__ void link_map(const Geom& g, LinkMap& m) {
    int tot = 0;
    for (int mu = 0; mu < 4; mu++) {
        int cnt = 1;
        for (int nu = 0; nu < 4; nu++) {
            int e = g.b[nu];
            if (nu == mu && g.nb[mu] != 1) e -= 1;
            m.ext[mu][nu] = e;
            cnt *= e;
        }
        m.off[mu] = tot;
        tot += cnt;
    }
    m.total = tot;
}

__device__ __forceinline__ int link_idx(const LinkMap& m, int mu, const int lc[4]) {
    return m.off[mu] + ((lc[0] * m.ext[mu][1] + lc[1]) * m.ext[mu][2] + lc[2]) * m.ext[mu][3] + lc[3];
}

// is the link (lc, mu) inside the block?  (a block spanning the lattice keeps its wrap link)
__device__ __forceinline__ bool link_internal(const Geom& g, int mu, const int lc[4]) {
    return g.nb[mu] == 1 || lc[mu] < g.b[mu] - 1;
}

template <class T>
__device__ __forceinline__ void su3_rebuild(cx<T> u[9]) {
    // conj(a b - c d) as products and fused multiply-adds
    auto cross = [](cx<T> a, cx<T> b, cx<T> c, cx<T> d) {
        cx<T> r = -(c * d);
        cmac(r, a, b);
        return conj(r);
    };
    u[6] = cross(u[1], u[5], u[2], u[4]);
    u[7] = cross(u[2], u[3], u[0], u[5]);
    u[8] = cross(u[0], u[4], u[1], u[3]);
}

template <class T>
__device__ __forceinline__ void lds_store(cx<T>* buf, int bvh, int l, const cx<T> v[12]) {
#pragma unroll
    for (int c = 0; c < 12; c++) buf[c * bvh + l] = v[c];
}

// hop k of the lane's own site (p, i) for the block residual.  tab[k][t]
// packs, for a hop inside the block, the LDS slot of the link (<< 8) and the
// neighbour's local index; -1 marks a hop that leaves the block (its link is
// read from memory).  The neighbour spinor comes from global memory psi.
template <class T, class S, class VP>
__device__ __forceinline__ void sap_hop(const FineOp<T, S>& op, int ltot, const cx<T>* __restrict__ L,
                                        const int* __restrict__ tab, int ntab, int k, int t, int p, int i,
                                        const int x[4], int base, const VP& psi, cx<T> acc[12]) {
    const Geom& g = op.g;
    const int code = tab[k * ntab + t];
    const int mu = k & 3;
    const bool fwd = k < 4;
    const int j = (code >= 0) ? base + (code & 255) : nb_index_sel(g, x, k);
    cx<T> v[12], u[9], h[6], gg[6];
    load_spinor(psi, g.vh, 1 - p, j, v);
    if (code >= 0) {
        const int li = code >> 8;
#pragma unroll
        for (int e = 0; e < 6; e++) u[e] = L[e * ltot + li];
        su3_rebuild(u);
    } else {
        load_link(op, fwd ? p : 1 - p, mu, fwd ? i : j, u);
    }
    const T sgn = fwd ? T(-1) : T(1);
    spin_project(mu, sgn, v, h);
    su3_two_spinor(u, !fwd, h, gg);
    spin_reconstruct(mu, sgn, gg, acc);
}

// value of the partner lane (lane ^ 1): DPP quad permutation [1, 0, 3, 2]
__device__ __forceinline__ float pair_swap(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// chirality half h (spins 2h, 2h + 1) of a spinor: global memory and the LDS block fields
template <class T>
__device__ __forceinline__ void half_load(const cx<T>* psi, int vh, int p, int h, int i, cx<T> v[6]) {
    const cx<T>* base = psi + (size_t)(p * 12 + 6 * h) * vh + i;
#pragma unroll
    for (int c = 0; c < 6; c++) v[c] = base[(size_t)c * vh];
}
template <class T>
__device__ __forceinline__ void half_store(cx<T>* psi, int vh, int p, int h, int i, const cx<T> v[6]) {
    cx<T>* base = psi + (size_t)(p * 12 + 6 * h) * vh + i;
#pragma unroll
    for (int c = 0; c < 6; c++) base[(size_t)c * vh] = v[c];
}
template <class T>
__device__ __forceinline__ void lds_load6(const cx<T>* buf, int bvh, int h, int l, cx<T> v[6]) {
#pragma unroll
    for (int c = 0; c < 6; c++) v[c] = buf[(6 * h + c) * bvh + l];
}
template <class T>
__device__ __forceinline__ void lds_store6(cx<T>* buf, int bvh, int h, int l, const cx<T> v[6]) {
#pragma unroll
    for (int c = 0; c < 6; c++) buf[(6 * h + c) * bvh + l] = v[c];
}
template <class T, class S>
__device__ __forceinline__ void clover_half_regs(const S* __restrict__ cl, int vh, int p, int h, int i, T m[36]) {
    const S* base = cl + (size_t)(p * 72 + h * 36) * vh + i;
#pragma unroll
    for (int r = 0; r < 36; r++) m[r] = T(base[(size_t)r * vh]);
}

// One block-internal hop of a site for the pair lane of chirality half h, in
// direction mu = 2h + Q, forward (FWD: neighbour x + mu, link U_mu(x), factor
// I - gamma_mu) or backward (x - mu, U_mu(x - mu)^H, I + gamma_mu).  With the
// chiral gamma matrices of dd_common.h the projection is h = psi_up + s B_mu
// psi_lo and the result (g, s B_mu^H g), g = U h, s = -1 forward, +1 backward.
// For the two directions of one lane the lower spin that feeds h_0 is the same
// (lo_1 on lane 0: mu = 0, 1; lo_0 on lane 1: mu = 2, 3), read at LDS offset
// oa (the other one at ob), and the remaining differences between B_0 / B_2
// and B_1 / B_3 are one sign, tau = +1 on lane 0 and -1 on lane 1:
//   Q = 0:  h_0 = u_0 + s i La,       h_1 = u_1 + s tau i Lb,
//           X  += s (-i) g_0,         Y  += s tau (-i) g_1,
//   Q = 1:  h_0 = u_0 - s tau La,     h_1 = u_1 + s Lb,
//           X  += -s tau g_0,         Y  += s g_1,
// where X is the lower spin fed by g_0 (lo_1 on lane 0, lo_0 on lane 1) and Y
// the one fed by g_1; up collects g itself.  code: the hop-table entry (LDS
// slot of the link << 8 | neighbour's local index), -1 for a hop that leaves
// the block.
template <class T, int Q, bool FWD>
__device__ __forceinline__ void pair_hop(const cx<T>* __restrict__ L, int ltot, int code, const cx<T>* buf, int bvh,
                                         int oa, int ob, T tau, cx<T> up[6], cx<T> X[3], cx<T> Y[3]) {
    if (code < 0) return;
    const int j = code & 255, li = code >> 8;
    cx<T> u[9];
#pragma unroll
    for (int e = 0; e < 6; e++) u[e] = L[e * ltot + li];
    su3_rebuild(u);
    const T s = FWD ? T(-1) : T(1);
    const T st = s * tau;
    cx<T> hv[6];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cx<T> u0 = buf[c * bvh + j], u1 = buf[(3 + c) * bvh + j];
        const cx<T> la = buf[oa + c * bvh + j], lb = buf[ob + c * bvh + j];
        if (Q == 0) {
            hv[c] = {u0.re - s * la.im, u0.im + s * la.re};
            hv[3 + c] = {u1.re - st * lb.im, u1.im + st * lb.re};
        } else {
            hv[c] = {u0.re - st * la.re, u0.im - st * la.im};
            hv[3 + c] = {u1.re + s * lb.re, u1.im + s * lb.im};
        }
    }
    cx<T> gv[6];
    su3_two_spinor(u, !FWD, hv, gv);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        up[c] += gv[c];
        up[3 + c] += gv[3 + c];
        if (Q == 0) {
            X[c] += cx<T>{s * gv[c].im, -s * gv[c].re};
            Y[c] += cx<T>{st * gv[3 + c].im, -st * gv[3 + c].re};
        } else {
            X[c] -= st * gv[c];
            Y[c] += s * gv[3 + c];
        }
    }
}

// MINW: waves per SIMD the register allocation must allow (2 for FP32 fields,
// so that two workgroups share a CU; FP64 needs the whole register file)
template <class T, class S, class VP, int MINW = (sizeof(T) > 4 ? 1 : 2)>
__global__ void __launch_bounds__(256, MINW) k_sap_fine(FineOp<T, S> op, const int* __restrict__ blocks, VP b0, VP z0,
                                                  int mr_steps, int nr, long ld, Mask mk) {
    extern __shared__ char smem_raw[];
    const Geom g = op.g;
    const int bvh = g.bvh;
    const int ntab = 2 * bvh;
    LinkMap lm;
    link_map(g, lm);
    const int ltot = lm.total;
    cx<T>* L = reinterpret_cast<cx<T>*>(smem_raw);  // [6][ltot] first two rows of internal links
    cx<T>* E = L + 6 * ltot;                         // even field [12][bvh]
    cx<T>* O = E + 12 * bvh;                         // odd field [12][bvh]
    int* tab = reinterpret_cast<int*>(O + 12 * bvh);  // [8][2 bvh] packed hop table, column p bvh + l
    double* red = reinterpret_cast<double*>(tab + 8 * ntab);
    const int blk = blocks[(op.sched & SCHED_XCD) ? xcd_swizzle(blockIdx.x, gridDim.x) : blockIdx.x];
    const int base = blk << g.lbvh;
    // Lanes 2l and 2l + 1 form a pair that owns the even site l and the odd
    // site l of the block.  Lane h holds chirality half h (spins 2h, 2h + 1) of
    // both sites' block vectors and of both clover blocks, so every clover
    // product and MR update is local to the lane; a hopping sum is split over
    // the pair by direction (lane h: mu = 2h, 2h + 1) and the halves meet
    // through one lane swap.  Only the residual, with its hops to other blocks,
    // is computed per site (lane h: the site of parity h).
    const int t = threadIdx.x;
    const bool act = t < 2 * bvh;
    const int h = t & 1;
    const int l = act ? t >> 1 : 0;
    const int i = base + l;
    const int sidx = h * bvh + l;
    int x[4];
    cb_coords(g, h, i, x);
    if (act) {
        int lc[4];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) lc[mu] = x[mu] & (g.b[mu] - 1);
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int mu = k & 3;
            int y[4];
            nb_coords(g, x, k, y);
            const int j = cb_index(g, y);
            int slot = -1;
            if ((j >> g.lbvh) == blk) {  // link joins two sites of the block
                int lo[4] = {lc[0], lc[1], lc[2], lc[3]};
                if (k >= 4) lo[mu] = (lc[mu] == 0) ? g.b[mu] - 1 : lc[mu] - 1;
                slot = link_idx(lm, mu, lo);
            }
            tab[k * ntab + sidx] = (slot >= 0) ? ((slot << 8) | (j - base)) : -1;
            // own forward link inside the block -> LDS (two rows)
            if (k < 4 && slot >= 0) {
                const cx<S>* src = op.U + (size_t)(h * 4 + mu) * 9 * g.vh + i;
#pragma unroll
                for (int e = 0; e < 6; e++) L[e * ltot + slot] = ccast<T>(src[(size_t)e * g.vh]);
            }
        }
    }
    // chirality half h of the clover blocks: A^{-1} at the even site, A at the odd site
    T me[36], mo[36];
    clover_half_regs(op.clovinv, g.vh, 0, h, i, me);
    clover_half_regs(op.clov, g.vh, 1, h, i, mo);
    __syncthreads();
    const int lane = t & 63, wv = t >> 6, nw = (blockDim.x + 63) >> 6;
    const T tau = h ? T(-1) : T(1);
    const int oa = (h ? 6 : 9) * bvh, ob = (h ? 9 : 6) * bvh;
    // chirality half h of the block-internal hopping sum at the site (P, l)
    // over the field buf (the neighbours' parity)
    auto pair_hops = [&](int P, const cx<T>* buf, cx<T> R[6]) {
        cx<T> up[6], X[3], Y[3];
#pragma unroll
        for (int c = 0; c < 6; c++) up[c] = czero<T>();
#pragma unroll
        for (int c = 0; c < 3; c++) X[c] = Y[c] = czero<T>();
        const int* tp = tab + P * bvh + l;
        const int d0 = 2 * h;
        pair_hop<T, 0, true>(L, ltot, tp[d0 * ntab], buf, bvh, oa, ob, tau, up, X, Y);
        pair_hop<T, 0, false>(L, ltot, tp[(4 + d0) * ntab], buf, bvh, oa, ob, tau, up, X, Y);
        pair_hop<T, 1, true>(L, ltot, tp[(1 + d0) * ntab], buf, bvh, oa, ob, tau, up, X, Y);
        pair_hop<T, 1, false>(L, ltot, tp[(5 + d0) * ntab], buf, bvh, oa, ob, tau, up, X, Y);
        // lane 0 keeps the upper spins and sends its lower-spin parts in the
        // order (lo_0, lo_1) = (Y, X); lane 1 keeps (lo_0, lo_1) = (X, Y) and
        // sends its upper spins
        cx<T> snd[6];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            snd[c] = h ? up[c] : Y[c];
            snd[3 + c] = h ? up[3 + c] : X[c];
        }
#pragma unroll
        for (int c = 0; c < 6; c++) {
            const cx<T> keep = h ? (c < 3 ? X[c] : Y[c - 3]) : up[c];
            R[c] = {keep.re + pair_swap(snd[c].re), keep.im + pair_swap(snd[c].im)};
        }
    };
    for (int rhs = 0; rhs < nr; rhs++) {
    if (!mk.on(rhs)) continue;
    const typename vrestrict<VP>::type b = b0 + rhs * ld;
    const typename vrestrict<VP>::type z = z0 + rhs * ld;
    // half h of: e_o, rho (the odd MR residual), w, R
    cx<T> eo[6], rho[6], w[6], R[6];
    // ---- residual on the block, b - H z with all 8 hops of the lane's own site ----
    if (act) {
        cx<T> acc[12], v[12];
#pragma unroll
        for (int c = 0; c < 12; c++) acc[c] = czero<T>();
#pragma unroll 1
        for (int k = 0; k < 8; k++) sap_hop<T, S>(op, ltot, L, tab, ntab, k, sidx, h, i, x, base, z, acc);
        load_spinor(b, g.vh, h, i, v);
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] += T(0.5) * acc[c];
        lds_store(h ? O : E, bvh, l, v);
    }
    __syncthreads();
    if (act) {
        cx<T> vh6[6], zh[6], t0[6];
        // t0_e = A_e^{-1} (b - H z)_e - z_e
        lds_load6(E, bvh, h, l, vh6);
        half_load(z, g.vh, 0, h, i, zh);
        herm6_apply(me, vh6, t0);
#pragma unroll
        for (int c = 0; c < 6; c++) {
            t0[c] -= zh[c];
            zh[c] += t0[c];
        }
        // z_e + t0 now (the block's z has been read by all its lanes), the
        // rest of e_e after the MR steps: t0 need not stay in registers
        half_store(z, g.vh, 0, h, i, zh);
        // r_o = (b - H z)_o - A_o z_o
        lds_load6(O, bvh, h, l, vh6);
        half_load(z, g.vh, 1, h, i, zh);
        herm6_apply(mo, zh, w);
#pragma unroll
        for (int c = 0; c < 6; c++) rho[c] = vh6[c] - w[c];
        lds_store6(E, bvh, h, l, t0);  // each lane overwrites only the half it read
    }
    __syncthreads();
    if (act) {
        // rho = f_o = r_o - D_oe t0, e_o = 0
        pair_hops(1, E, R);
#pragma unroll
        for (int c = 0; c < 6; c++) {
            rho[c] += T(0.5) * R[c];
            eo[c] = czero<T>();
        }
        lds_store6(O, bvh, h, l, rho);
    }
    __syncthreads();
    for (int it = 0; it < mr_steps; it++) {
        // even: w_e = A_e^{-1} (H_int rho), H = -1/2 hopsum
        if (act) {
            pair_hops(0, O, R);
#pragma unroll
            for (int c = 0; c < 6; c++) R[c] = T(-0.5) * R[c];
            herm6_apply(me, R, w);
            lds_store6(E, bvh, h, l, w);
        }
        __syncthreads();
        // odd: w_o = A_o rho - H_int w_e
        double sr = 0, si = 0, ss = 0;
        if (act) {
            pair_hops(1, E, R);
            herm6_apply(mo, rho, w);
#pragma unroll
            for (int c = 0; c < 6; c++) {
                w[c] += T(0.5) * R[c];
                cx<T> d = cmulc(w[c], rho[c]);
                sr += d.re;
                si += d.im;
                ss += norm2(w[c]);
            }
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        ss = wave_sum(ss);
        if (lane == 0) { red[3 * wv] = sr; red[3 * wv + 1] = si; red[3 * wv + 2] = ss; }
        __syncthreads();
        sr = si = ss = 0;
        for (int q = 0; q < nw; q++) { sr += red[3 * q]; si += red[3 * q + 1]; ss += red[3 * q + 2]; }
        if (act && ss > 0) {
            cx<T> alpha = {T(sr / ss), T(si / ss)};
#pragma unroll
            for (int c = 0; c < 6; c++) {
                eo[c] += alpha * rho[c];
                rho[c] -= alpha * w[c];
            }
        }
        // (two calls, not a pointer select: selecting between the arrays would
        // force both out of registers)
        if (act) {
            if (it + 1 < mr_steps) lds_store6(O, bvh, h, l, rho);
            else lds_store6(O, bvh, h, l, eo);
        }
        __syncthreads();
    }
    if (mr_steps == 0) {
        if (act) lds_store6(O, bvh, h, l, eo);
        __syncthreads();
    }
    // ---- back-substitution and update: e_e = t0 - A_e^{-1} (H_int e_o)_e, t0 already in z ----
    if (act) {
        pair_hops(0, O, R);
#pragma unroll
        for (int c = 0; c < 6; c++) R[c] = T(0.5) * R[c];
        herm6_apply(me, R, w);
        cx<T> zh[6];
        half_load(z, g.vh, 0, h, i, zh);
#pragma unroll
        for (int c = 0; c < 6; c++) zh[c] += w[c];
        half_store(z, g.vh, 0, h, i, zh);
        half_load(z, g.vh, 1, h, i, zh);
#pragma unroll
        for (int c = 0; c < 6; c++) zh[c] += eo[c];
        half_store(z, g.vh, 1, h, i, zh);
    }
    __syncthreads();  // the block fields are reused by the next right-hand side
    }
}

template <class T>
size_t fine_sap_lds_bytes(const Geom& g) {
    LinkMap lm;
    link_map(g, lm);
    int nt = ((2 * g.bvh + 63) / 64) * 64;
    return (6 * (size_t)lm.total + 24 * (size_t)g.bvh) * sizeof(cx<T>) + 8 * 2 * (size_t)g.bvh * sizeof(int) +
           3 * sizeof(double) * (nt / 64);
}

template <class T, class S, class VP>
static void sap_launch(const FineOp<T, S>& op, const int* blocks, int nblocks, VP b, VP z, int mr_steps, hipStream_t s,
                       int nr, long ld, Mask mk) {
    if (nblocks <= 0) return;
    int nt = ((2 * op.g.bvh + 63) / 64) * 64;
    size_t lds = fine_sap_lds_bytes<T>(op.g);
    static std::mutex mu;
    static size_t configured = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        // a refusal leaves its error for the launch below to report
        if (lds > 65536 && lds > configured &&
            hipFuncSetAttribute((const void*)k_sap_fine<T, S, VP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) == hipSuccess)
            configured = lds;
    }
    k_sap_fine<T, S, VP><<<nblocks, nt, lds, s>>>(op, blocks, b, z, mr_steps, nr, ld, mk);
}

template <class T, class S>
void fine_sap_half(const FineOp<T, S>& op, const int* blocks, int nblocks, const cx<T>* b, cx<T>* z, int mr_steps,
                   hipStream_t s, int nr, long ld, Mask mk) {
    sap_launch<T, S, cx<T>*>(op, blocks, nblocks, const_cast<cx<T>*>(b), z, mr_steps, s, nr, ld, mk);
}

template <class S>
void fine_sap_half_h(const FineOp<float, S>& op, const int* blocks, int nblocks, hspin b, hspin z, int mr_steps,
                     hipStream_t s, int nr, long ld, Mask mk) {
    sap_launch<float, S, hspin>(op, blocks, nblocks, b, z, mr_steps, s, nr, ld, mk);
}

// ---------------------------------------------------------------------------
// aggregation: coarse site gc (layout) owns the fine sites xc*a + l
// ---------------------------------------------------------------------------
__device__ __forceinline__ void agg_site(const AggMap& m, const int xc[4], int s, int x[4]) {
    int l3 = s % m.a[3]; s /= m.a[3];
    int l2 = s % m.a[2]; s /= m.a[2];
    int l1 = s % m.a[1];
    int l0 = s / m.a[1];
    x[0] = xc[0] * m.a[0] + l0;
    x[1] = xc[1] * m.a[1] + l1;
    x[2] = xc[2] * m.a[2] + l2;
    x[3] = xc[3] * m.a[3] + l3;
}

__device__ __forceinline__ void coarse_of(const AggMap& m, const int x[4], int xc[4]) {
    for (int mu = 0; mu < 4; mu++) xc[mu] = x[mu] / m.a[mu];
}

// sum of per-wave partials: lane 0 of each wave stores; after a sync thread 0..n-1 adds them up
// out[k] for k < n: P^H in, 2N unknowns per coarse site (index h*N + k)
// NT: the largest workgroup the build allows (one thread per aggregate site);
// the 256-thread form keeps two test vectors' loads in flight without spilling
template <class T, class S, int NT, class VI>
__global__ void __launch_bounds__(NT) k_restrict_fine(AggMap m, int N, const cx<S>* __restrict__ P, VI in0,
                                                      cx<T>* __restrict__ out, long ldi, long ldo, Mask mk) {
    if (!mk.on(blockIdx.y)) return;
    const VI in = in0 + blockIdx.y * ldi;
    out += blockIdx.y * ldo;
    extern __shared__ char smem_raw[];
    cx<double>* red = reinterpret_cast<cx<double>*>(smem_raw);  // [nw][2N]
    const int gc = blockIdx.x;
    const int pc = gc >= m.c.vh, ic = gc - pc * m.c.vh;
    int xc[4];
    cb_coords(m.c, pc, ic, xc);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
    const bool act = t < m.asz;
    int p = 0, i = 0;
    cx<T> v[12];
#pragma unroll
    for (int c = 0; c < 12; c++) v[c] = czero<T>();   // lanes past the aggregate add zeros
    if (act) {
        int x[4];
        agg_site(m, xc, t, x);
        p = site_parity(x);
        i = cb_index(m.f, x);
        load_spinor(in, m.f.vh, p, i, v);
    }
    const int vh = m.f.vh;
    // this workgroup's test vectors: [k0, k1) (the grid's z index splits them
    // when there are few coarse sites, so that enough workgroups stream P)
    const int kper = (N + gridDim.z - 1) / gridDim.z;
    const int k0 = blockIdx.z * kper, k1 = min(N, k0 + kper);
    // two test vectors at a time: both loads in flight before the reductions
    for (int k = k0; k < k1; k += 2) {
        const bool two = k + 1 < k1;
        cx<T> q[2][12];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            if (act && (u == 0 || two)) load_spinor(P + (size_t)(k + u) * 24 * vh, vh, p, i, q[u]);
            else
#pragma unroll
                for (int c = 0; c < 12; c++) q[u][c] = czero<T>();
        }
#pragma unroll
        for (int u = 0; u < 2; u++) {
            cx<double> d0 = czero<double>(), d1 = czero<double>();
#pragma unroll
            for (int c = 0; c < 6; c++) d0 += ccast<double>(cmulc(q[u][c], v[c]));
#pragma unroll
            for (int c = 6; c < 12; c++) d1 += ccast<double>(cmulc(q[u][c], v[c]));
            d0.re = wave_sum(d0.re); d0.im = wave_sum(d0.im);
            d1.re = wave_sum(d1.re); d1.im = wave_sum(d1.im);
            if (lane == 0 && (u == 0 || two)) { red[w * 2 * N + k + u] = d0; red[w * 2 * N + N + k + u] = d1; }
        }
    }
    __syncthreads();
    const int kn = max(0, k1 - k0);
    for (int e = t; e < 2 * kn; e += blockDim.x) {
        const int q = (e < kn) ? k0 + e : N + k0 + (e - kn);
        cx<double> s = czero<double>();
        for (int ww = 0; ww < nw; ww++) s += red[ww * 2 * N + q];
        out[(size_t)gc * 2 * N + q] = ccast<T>(s);
    }
}

template <class T, class S, class VO>
__global__ void k_prolong_fine(AggMap m, int N, const cx<S>* __restrict__ P, const cx<T>* __restrict__ in,
                               VO out0, long ldi, long ldo, Mask mk) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int vh = m.f.vh;
    if (gid >= 2 * vh || !mk.on(blockIdx.y)) return;
    in += blockIdx.y * ldi;
    const VO out = out0 + blockIdx.y * ldo;
    int p = gid >= vh, i = gid - p * vh;
    int x[4], xc[4];
    cb_coords(m.f, p, i, x);
    coarse_of(m, x, xc);
    int pc = lay_parity(m.c, xc), ic = cb_index(m.c, xc);
    const cx<T>* e = in + ((size_t)pc * m.c.vh + ic) * 2 * N;
    cx<T> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = czero<T>();
    for (int k = 0; k < N; k++) {
        cx<T> q[12];
        load_spinor(P + (size_t)k * 24 * vh, vh, p, i, q);
        cx<T> e0 = e[k], e1 = e[N + k];
#pragma unroll
        for (int c = 0; c < 6; c++) acc[c] += q[c] * e0;
#pragma unroll
        for (int c = 6; c < 12; c++) acc[c] += q[c] * e1;
    }
    store_spinor(out, vh, p, i, acc);
}

// Restriction and prolongation for a group of KR right-hand sides: every
// entry of P loaded from memory serves the whole group (P, N fine vectors, is
// the bulk of the traffic).  Per RHS the sums are formed in the same order as
// in the one-RHS kernels above.  Members of the group past the batch read the
// first member's data and are never stored.
template <class T, class S, int NT, int KR, class VI>
__global__ void __launch_bounds__(NT) k_restrict_fine_k(AggMap m, int N, const cx<S>* __restrict__ P, VI in,
                                                        cx<T>* __restrict__ out, long ldi, long ldo, int nr, Mask mk) {
    const int q0 = blockIdx.y * KR;
    bool on[KR];
    bool any = false;
    size_t io[KR];
#pragma unroll
    for (int r = 0; r < KR; r++) {
        on[r] = (q0 + r < nr) && mk.on(q0 + r);
        any |= on[r];
        io[r] = (size_t)(q0 + ((q0 + r < nr) ? r : 0)) * ldi;
    }
    if (!any) return;
    extern __shared__ char smem_raw[];
    cx<double>* red = reinterpret_cast<cx<double>*>(smem_raw);  // [nw][KR][2N]
    const int gc = blockIdx.x;
    const int pc = gc >= m.c.vh, ic = gc - pc * m.c.vh;
    int xc[4];
    cb_coords(m.c, pc, ic, xc);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
    const bool act = t < m.asz;
    int p = 0, i = 0;
    cx<T> v[KR][12];
#pragma unroll
    for (int r = 0; r < KR; r++)
#pragma unroll
        for (int c = 0; c < 12; c++) v[r][c] = czero<T>();
    if (act) {
        int x[4];
        agg_site(m, xc, t, x);
        p = site_parity(x);
        i = cb_index(m.f, x);
#pragma unroll
        for (int r = 0; r < KR; r++) load_spinor(in + io[r], m.f.vh, p, i, v[r]);
    }
    const int vh = m.f.vh;
    const int kper = (N + gridDim.z - 1) / gridDim.z;
    const int k0 = blockIdx.z * kper, k1 = min(N, k0 + kper);
    const int W = KR * 2 * N;   // reduction slots per wave
    for (int k = k0; k < k1; k++) {
        cx<T> q[12];
        if (act) load_spinor(P + (size_t)k * 24 * vh, vh, p, i, q);
        else
#pragma unroll
            for (int c = 0; c < 12; c++) q[c] = czero<T>();
#pragma unroll
        for (int r = 0; r < KR; r++) {
            cx<double> d0 = czero<double>(), d1 = czero<double>();
#pragma unroll
            for (int c = 0; c < 6; c++) d0 += ccast<double>(cmulc(q[c], v[r][c]));
#pragma unroll
            for (int c = 6; c < 12; c++) d1 += ccast<double>(cmulc(q[c], v[r][c]));
            d0.re = wave_sum(d0.re); d0.im = wave_sum(d0.im);
            d1.re = wave_sum(d1.re); d1.im = wave_sum(d1.im);
            if (lane == 0) { red[w * W + r * 2 * N + k] = d0; red[w * W + r * 2 * N + N + k] = d1; }
        }
    }
    __syncthreads();
    const int kn = max(0, k1 - k0);
    for (int e = t; e < KR * 2 * kn; e += blockDim.x) {
        const int r = e / (2 * kn), e2 = e % (2 * kn);
        if (!on[r]) continue;
        const int q = (e2 < kn) ? k0 + e2 : N + k0 + (e2 - kn);
        cx<double> sum = czero<double>();
        for (int ww = 0; ww < nw; ww++) sum += red[ww * W + r * 2 * N + q];
        out[(size_t)(q0 + r) * ldo + (size_t)gc * 2 * N + q] = ccast<T>(sum);
    }
}

template <class T, class S, int KR, class VO>
__global__ void __launch_bounds__(256) k_prolong_fine_k(AggMap m, int N, const cx<S>* __restrict__ P, const cx<T>* __restrict__ in,
                                 VO out, long ldi, long ldo, int nr, Mask mk) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int vh = m.f.vh;
    if (gid >= 2 * vh) return;
    const int q0 = blockIdx.y * KR;
    bool on[KR];
    bool any = false;
    size_t io[KR];
#pragma unroll
    for (int r = 0; r < KR; r++) {
        on[r] = (q0 + r < nr) && mk.on(q0 + r);
        any |= on[r];
        io[r] = (size_t)(q0 + ((q0 + r < nr) ? r : 0)) * ldi;
    }
    if (!any) return;
    int p = gid >= vh, i = gid - p * vh;
    int x[4], xc[4];
    cb_coords(m.f, p, i, x);
    coarse_of(m, x, xc);
    int pc = lay_parity(m.c, xc), ic = cb_index(m.c, xc);
    const size_t eo = ((size_t)pc * m.c.vh + ic) * 2 * N;
    cx<T> acc[KR][12];
#pragma unroll
    for (int r = 0; r < KR; r++)
#pragma unroll
        for (int c = 0; c < 12; c++) acc[r][c] = czero<T>();
    for (int k = 0; k < N; k++) {
        cx<T> q[12];
        load_spinor(P + (size_t)k * 24 * vh, vh, p, i, q);
#pragma unroll
        for (int r = 0; r < KR; r++) {
            const cx<T> e0 = in[io[r] + eo + k], e1 = in[io[r] + eo + N + k];
#pragma unroll
            for (int c = 0; c < 6; c++) acc[r][c] += q[c] * e0;
#pragma unroll
            for (int c = 6; c < 12; c++) acc[r][c] += q[c] * e1;
        }
    }
#pragma unroll
    for (int r = 0; r < KR; r++)
        if (on[r]) store_spinor(out + (size_t)(q0 + r) * ldo, vh, p, i, acc[r]);
}

// group size for a batch of nr right-hand sides (FP64 fields hold twice the
// registers, so their groups are half as large)
template <class T> static int transfer_group(int nr) {
    const int cap = sizeof(T) == 8 ? 2 : 4;
    return nr >= cap ? cap : (nr >= 2 ? 2 : 1);
}

template <class T, class S, class VI>
static void restrict_launch(const AggMap& m, int N, const cx<S>* P, VI in, cx<T>* out, hipStream_t s, int nr,
                            long ldi, long ldo, Mask mk) {
    int nt = ((m.asz + 63) / 64) * 64;
    // split the test vectors over workgroups until about 1024 stream P
    const int ks = std::max(1, std::min(N, (1024 + 2 * m.c.vh - 1) / (2 * m.c.vh)));
    const int kr = transfer_group<T>(nr);
    if (kr == 1 || nt > 256) {
        size_t lds = sizeof(cx<double>) * 2 * N * (nt / 64);
        dim3 grid(2 * m.c.vh, nr, ks);
        if (nt <= 256) k_restrict_fine<T, S, 256, VI><<<grid, nt, lds, s>>>(m, N, P, in, out, ldi, ldo, mk);
        else k_restrict_fine<T, S, 1024, VI><<<grid, nt, lds, s>>>(m, N, P, in, out, ldi, ldo, mk);
        return;
    }
    size_t lds = sizeof(cx<double>) * kr * 2 * N * (nt / 64);
    dim3 grid(2 * m.c.vh, (nr + kr - 1) / kr, ks);
    if constexpr (sizeof(T) == 4)
        if (kr == 4) {
            k_restrict_fine_k<T, S, 256, 4, VI><<<grid, nt, lds, s>>>(m, N, P, in, out, ldi, ldo, nr, mk);
            return;
        }
    k_restrict_fine_k<T, S, 256, 2, VI><<<grid, nt, lds, s>>>(m, N, P, in, out, ldi, ldo, nr, mk);
}
template <class T, class S, class VO>
static void prolong_launch(const AggMap& m, int N, const cx<S>* P, const cx<T>* in, VO out, hipStream_t s, int nr,
                           long ldi, long ldo, Mask mk) {
    const int kr = transfer_group<T>(nr);
    if (kr == 1) {
        dim3 grid(nblk_of(2L * m.f.vh, 256), nr);
        k_prolong_fine<T, S, VO><<<grid, 256, 0, s>>>(m, N, P, in, out, ldi, ldo, mk);
        return;
    }
    dim3 grid(nblk_of(2L * m.f.vh, 256), (nr + kr - 1) / kr);
    if constexpr (sizeof(T) == 4)
        if (kr == 4) {
            k_prolong_fine_k<T, S, 4, VO><<<grid, 256, 0, s>>>(m, N, P, in, out, ldi, ldo, nr, mk);
            return;
        }
    k_prolong_fine_k<T, S, 2, VO><<<grid, 256, 0, s>>>(m, N, P, in, out, ldi, ldo, nr, mk);
}

template <class T, class S>
void fine_restrict(const AggMap& m, int N, const cx<S>* P, const cx<T>* in, cx<T>* out, hipStream_t s, int nr,
                   long ldi, long ldo, Mask mk) {
    restrict_launch<T, S, const cx<T>*>(m, N, P, in, out, s, nr, ldi, ldo, mk);
}
template <class T, class S>
void fine_prolong(const AggMap& m, int N, const cx<S>* P, const cx<T>* in, cx<T>* out, hipStream_t s, int nr,
                  long ldi, long ldo, Mask mk) {
    prolong_launch<T, S, cx<T>*>(m, N, P, in, out, s, nr, ldi, ldo, mk);
}
template <class S>
void fine_restrict_h(const AggMap& m, int N, const cx<S>* P, hspin in, cx<float>* out, hipStream_t s, int nr, long ldi,
                     long ldo, Mask mk) {
    restrict_launch<float, S, hspin>(m, N, P, in, out, s, nr, ldi, ldo, mk);
}
template <class S>
void fine_prolong_h(const AggMap& m, int N, const cx<S>* P, const cx<float>* in, hspin out, hipStream_t s, int nr,
                    long ldi, long ldo, Mask mk) {
    prolong_launch<float, S, hspin>(m, N, P, in, out, s, nr, ldi, ldo, mk);
}

// ---------------------------------------------------------------------------
// FP16 spinor sets (hspin): conversion from and to FP64 / FP32 sets and the
// FGMRES update x += sum_j y_j Z_j, one thread per (parity, chirality half,
// site) -- the thread index is the scale's index
// ---------------------------------------------------------------------------
template <class S>
__global__ void k_hpack(int vh, const cx<S>* __restrict__ in, hspin out, long ld, Mask mk) {
    const long gid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (gid >= 4L * vh || !mk.on(blockIdx.y)) return;
    const int ph = (int)(gid / vh), i = (int)(gid - (long)ph * vh);
    const int p = ph >> 1, h = ph & 1;
    const cx<S>* src = in + blockIdx.y * ld + (size_t)(p * 12 + 6 * h) * vh + i;
    cx<float> v[6];
#pragma unroll
    for (int c = 0; c < 6; c++) v[c] = ccast<float>(src[(size_t)c * vh]);
    half_store(out + blockIdx.y * ld, vh, p, h, i, v);
}
template <class D>
__global__ void k_hunpack(int vh, hspin in, cx<D>* __restrict__ out, long ld, Mask mk) {
    const long gid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (gid >= 4L * vh || !mk.on(blockIdx.y)) return;
    const int ph = (int)(gid / vh), i = (int)(gid - (long)ph * vh);
    const int p = ph >> 1, h = ph & 1;
    cx<float> v[6];
    half_load(in + blockIdx.y * ld, vh, p, h, i, v);
    cx<D>* dst = out + blockIdx.y * ld + (size_t)(p * 12 + 6 * h) * vh + i;
#pragma unroll
    for (int c = 0; c < 6; c++) dst[(size_t)c * vh] = ccast<D>(v[c]);
}
__global__ void k_hlincomb(int vh, Counts mc, hspin Z, long ldz, const cx<double>* __restrict__ y,
                           cx<double>* __restrict__ x, long ldzr, int ystride, long ldx, Mask mk) {
    const long gid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (gid >= 4L * vh || !mk.on(blockIdx.y)) return;
    const int ph = (int)(gid / vh), i = (int)(gid - (long)ph * vh);
    const int p = ph >> 1, h = ph & 1;
    const int m = mc.v[blockIdx.y];
    const hspin z = Z + blockIdx.y * ldzr;
    y += (size_t)blockIdx.y * ystride;
    cx<double>* xp = x + blockIdx.y * ldx + (size_t)(p * 12 + 6 * h) * vh + i;
    cx<double> acc[6];
#pragma unroll
    for (int c = 0; c < 6; c++) acc[c] = xp[(size_t)c * vh];
    for (int j = 0; j < m; j++) {
        cx<float> v[6];
        half_load(z + (long)j * ldz, vh, p, h, i, v);
        const cx<double> yj = y[j];
#pragma unroll
        for (int c = 0; c < 6; c++) acc[c] += yj * ccast<double>(v[c]);
    }
#pragma unroll
    for (int c = 0; c < 6; c++) xp[(size_t)c * vh] = acc[c];
}

template <class S>
void fine_hpack(int vh, const cx<S>* in, hspin out, long ld, int nr, Mask mk, hipStream_t s) {
    dim3 grid(nblk_of(4L * vh, 256), nr);
    k_hpack<S><<<grid, 256, 0, s>>>(vh, in, out, ld, mk);
}
template <class D>
void fine_hunpack(int vh, hspin in, cx<D>* out, long ld, int nr, Mask mk, hipStream_t s) {
    dim3 grid(nblk_of(4L * vh, 256), nr);
    k_hunpack<D><<<grid, 256, 0, s>>>(vh, in, out, ld, mk);
}
void fine_hlincomb(int vh, int m, hspin Z, long ldz, const cx<double>* y, cx<double>* x, hipStream_t s, int nr,
                   long ldzr, int ystride, long ldx, Mask mk, const Counts* per) {
    Counts mc;
    for (int r = 0; r < MAX_RHS; r++) mc.v[r] = (per && r < nr) ? std::min(per->v[r], m) : m;
    dim3 grid(nblk_of(4L * vh, 256), nr);
    k_hlincomb<<<grid, 256, 0, s>>>(vh, mc, Z, ldz, y, x, ldzr, ystride, ldx, mk);
}

// ---------------------------------------------------------------------------
// local orthonormalisation: modified Gram-Schmidt of v_1..v_N restricted to
// one aggregate (coarse site gc, spin half h), in the order 1..N
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_gs_fine(AggMap m, int N, const cx<T>* __restrict__ tv, cx<T>* __restrict__ P, int* bad) {
    __shared__ double red[2 * 16];
    const int gc = blockIdx.x, h = blockIdx.y;
    const int pc = gc >= m.c.vh, ic = gc - pc * m.c.vh;
    int xc[4];
    cb_coords(m.c, pc, ic, xc);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
    const bool act = t < m.asz;
    const int vh = m.f.vh;
    int p = 0, i = 0;
    if (act) {
        int x[4];
        agg_site(m, xc, t, x);
        p = site_parity(x);
        i = cb_index(m.f, x);
    }
    for (int k = 0; k < N; k++) {
        cx<double> q[6];
        const size_t off_k = (size_t)k * 24 * vh + (size_t)(p * 12 + 6 * h) * vh + i;
#pragma unroll
        for (int c = 0; c < 6; c++) q[c] = act ? ccast<double>(tv[off_k + (size_t)c * vh]) : czero<double>();
        for (int j = 0; j < k; j++) {
            const size_t off_j = (size_t)j * 24 * vh + (size_t)(p * 12 + 6 * h) * vh + i;
            cx<T> pj[6];
            cx<double> d = czero<double>();
            if (act) {
#pragma unroll
                for (int c = 0; c < 6; c++) {
                    pj[c] = P[off_j + (size_t)c * vh];
                    d += cmulc(ccast<double>(pj[c]), q[c]);
                }
            }
            d.re = wave_sum(d.re);
            d.im = wave_sum(d.im);
            __syncthreads();
            if (lane == 0) { red[2 * w] = d.re; red[2 * w + 1] = d.im; }
            __syncthreads();
            d = czero<double>();
            for (int ww = 0; ww < nw; ww++) { d.re += red[2 * ww]; d.im += red[2 * ww + 1]; }
            if (act) {
#pragma unroll
                for (int c = 0; c < 6; c++) q[c] -= d * ccast<double>(pj[c]);
            }
        }
        double n2 = 0;
#pragma unroll
        for (int c = 0; c < 6; c++) n2 += norm2(q[c]);
        n2 = wave_sum(n2);
        __syncthreads();
        if (lane == 0) red[2 * w] = n2;
        __syncthreads();
        n2 = 0;
        for (int ww = 0; ww < nw; ww++) n2 += red[2 * ww];
        double inv = 0;
        if (n2 > 0) inv = 1.0 / sqrt(n2);
        else if (t == 0) atomicAdd(bad, 1);
        if (act) {
#pragma unroll
            for (int c = 0; c < 6; c++) P[off_k + (size_t)c * vh] = ccast<T>(inv * q[c]);
        }
    }
}

template <class T>
void fine_gram_schmidt(const AggMap& m, int N, const cx<T>* tv, cx<T>* P, int* bad, hipStream_t s) {
    int nt = ((m.asz + 63) / 64) * 64;
    dim3 grid(2 * m.c.vh, 2);
    k_gs_fine<T><<<grid, nt, 0, s>>>(m, N, tv, P, bad);
}

// ---------------------------------------------------------------------------
// D_c = P^H D P: workgroup (coarse site c, column b = hb*N + kb); slot 0
// collects the self coupling and the hops that stay inside the aggregate's
// lattice block, slot 1+k the hops k that leave it.  Accumulated in FP64.
// ---------------------------------------------------------------------------
// NT: the largest workgroup (one thread per aggregate site) the build allows;
// the 256-thread form has the register file to keep its state without scratch
template <class T, int NT>
__global__ void __launch_bounds__(NT) k_assemble_fine(FineOp<T> op, AggMap m, int N, const cx<T>* __restrict__ P,
                                                      cx<T>* __restrict__ M) {
    extern __shared__ char smem_raw[];
    cx<double>* red = reinterpret_cast<cx<double>*>(smem_raw);  // [nw][2N]
    // workgroup (coarse site gc, column bcol); the 2N workgroups of one coarse
    // site run back to back on one XCD, sharing its L2 for the aggregate's P
    const int nd = 2 * N;
    const int lw = xcd_swizzle(blockIdx.x, gridDim.x);
    const int gc = lw / nd, bcol = lw - gc * nd;
    const int hb = bcol / N, kb = bcol % N;
    const int pc = gc >= m.c.vh, ic = gc - pc * m.c.vh;
    int xc[4];
    cb_coords(m.c, pc, ic, xc);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
    const bool act = t < m.asz;
    const int vh = m.f.vh;
    int x[4] = {0, 0, 0, 0}, p = 0, i = 0;
    if (act) {
        agg_site(m, xc, t, x);
        p = site_parity(x);
        i = cb_index(m.f, x);
    }
    const cx<T>* Pb = P + (size_t)kb * 24 * vh;
    for (int slot = 0; slot < 9; slot++) {
        cx<T> wv[12];
#pragma unroll
        for (int c = 0; c < 12; c++) wv[c] = czero<T>();
        if (act) {
            if (slot == 0) {
                cx<T> v[12];
                load_spinor(Pb, vh, p, i, v);
#pragma unroll
                for (int c = 0; c < 12; c++)
                    if ((c / 6) != hb) v[c] = czero<T>();
                clover_apply(op.clov, vh, p, i, v, wv);
                cx<T> acc[12];
#pragma unroll
                for (int c = 0; c < 12; c++) acc[c] = czero<T>();
                for (int k = 0; k < 8; k++) {
                    int y[4], yc[4];
                    nb_coords(op.g, x, k, y);
                    coarse_of(m, y, yc);
                    if (yc[0] != xc[0] || yc[1] != xc[1] || yc[2] != xc[2] || yc[3] != xc[3]) continue;
                    int j = cb_index(op.g, y);
                    // opaque per iteration: keeps the compiler from hoisting the
                    // neighbour's addresses out of the slot loop (they would not
                    // fit in registers)
                    asm volatile("" : "+v"(j));
                    load_spinor(Pb, vh, 1 - p, j, v);
#pragma unroll
                    for (int c = 0; c < 12; c++)
                        if ((c / 6) != hb) v[c] = czero<T>();
                    hop_accum(op, k, p, i, j, v, acc);
                }
#pragma unroll
                for (int c = 0; c < 12; c++) wv[c] -= T(0.5) * acc[c];
            } else {
                int k = slot - 1;
                int y[4], yc[4];
                nb_coords(op.g, x, k, y);
                coarse_of(m, y, yc);
                if (yc[0] != xc[0] || yc[1] != xc[1] || yc[2] != xc[2] || yc[3] != xc[3]) {
                    int j = cb_index(op.g, y);
                    // opaque per iteration: keeps the compiler from hoisting the
                    // neighbour's addresses out of the slot loop (they would not
                    // fit in registers)
                    asm volatile("" : "+v"(j));
                    cx<T> v[12], acc[12];
                    load_spinor(Pb, vh, 1 - p, j, v);
#pragma unroll
                    for (int c = 0; c < 12; c++) {
                        if ((c / 6) != hb) v[c] = czero<T>();
                        acc[c] = czero<T>();
                    }
                    hop_accum(op, k, p, i, j, v, acc);
#pragma unroll
                    for (int c = 0; c < 12; c++) wv[c] = T(-0.5) * acc[c];
                }
            }
        }
        // projections onto the aggregate's columns a, AB at a time so that
        // their loads and reductions overlap
        constexpr int AB = 4;
        for (int a0 = 0; a0 < nd; a0 += AB) {
            cx<T> pa[AB][6];
#pragma unroll
            for (int u = 0; u < AB; u++) {
                const int a = a0 + u, ha = a / N, ka = a % N;
                const cx<T>* Pa = P + (size_t)ka * 24 * vh + (size_t)(p * 12 + 6 * ha) * vh + i;
#pragma unroll
                for (int c = 0; c < 6; c++) pa[u][c] = (act && a < nd) ? Pa[(size_t)c * vh] : czero<T>();
            }
            cx<double> d[AB];
#pragma unroll
            for (int u = 0; u < AB; u++) {
                const int ha = ((a0 + u) / N) & 1;
                d[u] = czero<double>();
#pragma unroll
                for (int c = 0; c < 6; c++) d[u] += cmulc(ccast<double>(pa[u][c]), ccast<double>(wv[6 * ha + c]));
            }
#pragma unroll
            for (int u = 0; u < AB; u++) {
                d[u].re = wave_sum(d[u].re);
                d[u].im = wave_sum(d[u].im);
            }
            if (lane == 0) {
#pragma unroll
                for (int u = 0; u < AB; u++)
                    if (a0 + u < nd) red[w * nd + a0 + u] = d[u];
            }
        }
        __syncthreads();
        for (int a = t; a < nd; a += blockDim.x) {
            cx<double> s = czero<double>();
            for (int ww = 0; ww < nw; ww++) s += red[ww * nd + a];
            M[(((size_t)gc * 9 + slot) * nd + bcol) * nd + a] = ccast<T>(s);  // column-major block
        }
        __syncthreads();
    }
}

template <class T>
void fine_assemble(const FineOp<T>& op, const AggMap& m, int N, const cx<T>* P, cx<T>* M, hipStream_t s) {
    int nt = ((m.asz + 63) / 64) * 64;
    size_t lds = sizeof(cx<double>) * 2 * N * (nt / 64);
    const int nwg = 2 * m.c.vh * 2 * N;
    if (nt <= 256) k_assemble_fine<T, 256><<<nwg, nt, lds, s>>>(op, m, N, P, M);
    else k_assemble_fine<T, 1024><<<nwg, nt, lds, s>>>(op, m, N, P, M);
}

// ---------------------------------------------------------------------------
// counter-based normal numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11) keyed by the seed, counter (element index, vector, stream), then the
// Box-Muller transform.  Element e of vector v gets re + i im ~ N(0,1) each.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ cx<double> gauss_pair(unsigned long long seed, unsigned long long e, int v, int sid) {
    uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), (uint32_t)v, (uint32_t)sid};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    double u1 = (c[0] + 0.5) * (1.0 / 4294967296.0);
    double u2 = (c[1] + 0.5) * (1.0 / 4294967296.0);
    double r = sqrt(-2.0 * log(u1));
    return {r * cos(2.0 * M_PI * u2), r * sin(2.0 * M_PI * u2)};
}

template <class T>
__global__ void k_random_fine(Geom g, int n, unsigned long long seed, int sid, cx<T>* out) {
    long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long vol = 2L * g.vh;
    if (s >= vol) return;
    int x[4];
    canon_coords(g.d, s, x);
    int p = site_parity(x), i = cb_index(g, x);
    for (int v = 0; v < n; v++)
        for (int c = 0; c < 12; c++)
            out[(size_t)v * 24 * g.vh + (size_t)(p * 12 + c) * g.vh + i] = ccast<T>(gauss_pair(seed, s * 12 + c, v, sid));
}

template <class T>
void fine_random(const Geom& g, int n, unsigned long long seed, int sid, cx<T>* out, hipStream_t s) {
    k_random_fine<T><<<nblk_of(2L * g.vh, 256), 256, 0, s>>>(g, n, seed, sid, out);
}

// ---------------------------------------------------------------------------
// operator kernels for compute type T and storage type S
#define DD_FINE_OP_INST(T, S)                                                                                 \
    template void fine_dirac<T, S>(const FineOp<T, S>&, const cx<T>*, cx<T>*, hipStream_t, int, long, Mask);  \
    template void fine_oe_hop<T, S>(const FineOp<T, S>&, int, bool, bool, double, double, const cx<T>*,         \
                                    const cx<T>*, cx<T>*, hipStream_t);                                       \
    template void fine_sap_half<T, S>(const FineOp<T, S>&, const int*, int, const cx<T>*, cx<T>*, int, hipStream_t, \
                                      int, long, Mask);                                                       \
    template void fine_restrict<T, S>(const AggMap&, int, const cx<S>*, const cx<T>*, cx<T>*, hipStream_t, int,   \
                                      long, long, Mask);                                                      \
    template void fine_prolong<T, S>(const AggMap&, int, const cx<S>*, const cx<T>*, cx<T>*, hipStream_t, int,    \
                                     long, long, Mask);

#define DD_FINE_INST(T)                                                                                      \
    template void fine_import_gauge<T>(const Geom&, const double*, cx<T>*, hipStream_t);                     \
    template void fine_import_spinor<T>(const Geom&, const double*, cx<T>*, hipStream_t);                    \
    template void fine_export_spinor<T>(const Geom&, const cx<T>*, double*, hipStream_t);                    \
    template void fine_import_vectors<T>(const Geom&, int, const double*, cx<T>*, hipStream_t);              \
    template void fine_export_vectors<T>(const Geom&, int, const cx<T>*, double*, hipStream_t);              \
    DD_FINE_OP_INST(T, T)                                                                                    \
    template void fine_gram_schmidt<T>(const AggMap&, int, const cx<T>*, cx<T>*, int*, hipStream_t);         \
    template void fine_assemble<T>(const FineOp<T>&, const AggMap&, int, const cx<T>*, cx<T>*, hipStream_t); \
    template void fine_random<T>(const Geom&, int, unsigned long long, int, cx<T>*, hipStream_t);            \
    template size_t fine_sap_lds_bytes<T>(const Geom&);

DD_FINE_INST(double)
DD_FINE_INST(float)
DD_FINE_OP_INST(float, _Float16)

// FP16 spinor sets (FP32 arithmetic) with FP32 or FP16 operator storage
#define DD_FINE_H_INST(S)                                                                                     \
    template void fine_sap_half_h<S>(const FineOp<float, S>&, const int*, int, hspin, hspin, int, hipStream_t, \
                                     int, long, Mask);                                                        \
    template void fine_restrict_h<S>(const AggMap&, int, const cx<S>*, hspin, cx<float>*, hipStream_t, int, long, \
                                     long, Mask);                                                             \
    template void fine_prolong_h<S>(const AggMap&, int, const cx<S>*, const cx<float>*, hspin, hipStream_t, int, \
                                    long, long, Mask);
DD_FINE_H_INST(float)
DD_FINE_H_INST(_Float16)
template void fine_hpack<double>(int, const cx<double>*, hspin, long, int, Mask, hipStream_t);
template void fine_hpack<float>(int, const cx<float>*, hspin, long, int, Mask, hipStream_t);
template void fine_hunpack<double>(int, hspin, cx<double>*, long, int, Mask, hipStream_t);
template void fine_hunpack<float>(int, hspin, cx<float>*, long, int, Mask, hipStream_t);

}  // namespace dd
