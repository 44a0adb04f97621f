// dd_coarse.hip -- kernels on coarse levels (nd = 2N unknowns per site).
//
//   coarse stencil D_c ............ nearest-neighbour blocks of P^H D P (Sec. 3.2)
//   odd-even pieces ............... Schur complement A_oo - D_oe A_ee^{-1} D_eo (Sec. 5)
//   self-block inverses ........... dense Gauss-Jordan in FP64
//   coarse SAP, P^H, P, Gram-Schmidt, assembly of the next coarser operator
//                                   (recursive application, Sec. 3 and 5)
//
// Vectors are [parity][layout index][nd] (a site's unknowns contiguous);
// operator blocks are column-major so that the thread owning row r reads
// consecutive addresses across the wavefront.
#include <stdexcept>
#include <type_traits>

#include "dd_kernels.h"

namespace dd {

static inline int nblk_of(long n, int b) { return (int)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// out(x) = [post Minv] ( self(x) in1(x) + hop_sign * sum_k M_{1+k}(x) in2(x_k) )
// One workgroup per site.  The site's blocks used here lie back to back in
// memory (self, then the 8 hops, each column-major), so (block, column) pair
// q is column q of one nd-row panel.  The pairs are split evenly over the
// wavefronts and lane r accumulates row r: every load is coalesced.  On small
// coarse lattices (a few hundred sites) the kernel is bound by memory latency,
// not bandwidth, so each lane issues the loads of its first pairs (and of its
// columns of the self-block inverse) before the site's input vectors
// (hop sign folded in) are staged in LDS: block entries and inputs are in
// flight together.  Partial rows meet in LDS.
// ---------------------------------------------------------------------------
static constexpr int CA_WAVES = 12;
// block entries and inverse-block columns a lane loads at once (fewer in
// FP64, where they take twice the registers)
template <class S> struct CaPre {
    static constexpr int N = sizeof(S) > 4 ? 24 : 30;
    static constexpr int INV = sizeof(S) > 4 ? 4 : 8;
};

template <class T, class S>
__global__ void __launch_bounds__(64 * CA_WAVES) k_coarse_apply(CoarseOp<T, S> op, int par, int self_mode,
                                                                const cx<T>* __restrict__ in1, int hop_sign,
                                                                const cx<T>* in2, int post_inv, cx<T>* out,
                                                                Mask mk, long ld) {
    if (!mk.on(blockIdx.y)) return;
    {
        const long off = blockIdx.y * ld;
        if (in1) in1 += off;
        if (in2) in2 += off;
        out += off;
    }
    __shared__ cx<T> part[CA_WAVES][64];
    __shared__ cx<T> X[9 * 64];            // staged inputs [slot][nd] (nd <= 64)
    __shared__ const cx<T>* vin[9];
    const Geom g = op.g;
    const int nd = op.nd;
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6, r = threadIdx.x & 63;
    int p, i;
    if (par < 0) { p = blockIdx.x >= g.vh; i = blockIdx.x - p * g.vh; }
    else { p = par; i = blockIdx.x; }
    const size_t gs = (size_t)p * g.vh + i;
    const size_t nn = (size_t)nd * nd;
    const int nself = (self_mode == CS_SELF || self_mode == CS_SELFINV) ? 1 : 0;
    // first block of the panel: the self block, its inverse, or the first hop
    const cx<S>* panel = (self_mode == CS_SELFINV) ? op.Minv + gs * nn : op.M + (gs * 9 + 1 - nself) * nn;
    // input vectors of the panel's column slots: thread k < 8 finds neighbour k
    if (threadIdx.x == 0 && nself) vin[0] = in1 + gs * nd;
    if (hop_sign != 0 && threadIdx.x < 8) {
        int x[4];
        cb_coords(g, p, i, x);
        vin[nself + threadIdx.x] = in2 + nb_global(g, p, x, threadIdx.x) * nd;
    }
    const int ns = nself + (hop_sign != 0 ? 8 : 0);
    const int Q = ns * nd;
    const int per = (Q + nw - 1) / nw;
    const int q0 = w * per, q1 = min(Q, q0 + per);
    const bool row = r < nd;
    const cx<S>* A = panel + r;
    constexpr int CA_PRE = CaPre<S>::N;
    cx<S> a[CA_PRE];
    auto load_pairs = [&](int qb) {
#pragma unroll
        for (int u = 0; u < CA_PRE; u++)
            a[u] = (row && qb + u < q1) ? A[(size_t)(qb + u) * nd] : cx<S>{S(0), S(0)};
    };
    load_pairs(q0);
    const int per2 = (nd + nw - 1) / nw;
    const int c0 = w * per2, c1 = min(nd, c0 + per2);
    const cx<S>* Ainv = op.Minv + gs * nn + r;
    constexpr int CA_INV = CaPre<S>::INV;
    cx<S> b[CA_INV];
    auto load_inv = [&](int cb) {
#pragma unroll
        for (int u = 0; u < CA_INV; u++)
            b[u] = (row && cb + u < c1) ? Ainv[(size_t)(cb + u) * nd] : cx<S>{S(0), S(0)};
    };
    if (post_inv) load_inv(c0);
    __syncthreads();
    for (int e = threadIdx.x; e < Q; e += blockDim.x) {
        const int s2 = e / nd;
        const cx<T> v = vin[s2][e - s2 * nd];
        X[e] = (s2 >= nself && hop_sign < 0) ? -v : v;
    }
    __syncthreads();
    cx<T> acc = czero<T>();
    for (int qb = q0; qb < q1; qb += CA_PRE) {
        if (qb != q0) load_pairs(qb);
#pragma unroll
        for (int u = 0; u < CA_PRE; u++)
            if (qb + u < q1) acc += ccast<T>(a[u]) * X[qb + u];
    }
    part[w][r] = acc;
    __syncthreads();
    cx<T> tot = czero<T>();
    if (w == 0 && row) {
        tot = (self_mode == CS_IDENT) ? in1[gs * nd + r] : czero<T>();
        for (int q = 0; q < nw; q++) tot += part[q][r];
    }
    if (!post_inv) {
        if (w == 0 && row) out[gs * nd + r] = tot;
        return;
    }
    if (w == 0) X[r] = tot;
    __syncthreads();
    cx<T> a3 = czero<T>();
    for (int cb = c0; cb < c1; cb += CA_INV) {
        if (cb != c0) load_inv(cb);
#pragma unroll
        for (int u = 0; u < CA_INV; u++)
            if (cb + u < c1) a3 += ccast<T>(b[u]) * X[cb + u];
    }
    part[w][r] = a3;
    __syncthreads();
    if (w == 0 && row) {
        cx<T> s2 = czero<T>();
        for (int q = 0; q < nw; q++) s2 += part[q][r];
        out[gs * nd + r] = s2;
    }
}

// ---------------------------------------------------------------------------
// Multi-RHS coarse stencil on the matrix cores.  For one site and k <= 16
// right-hand sides the apply is a sum of complex products
//     C (nd x k) += M_s (nd x nd) X_s (nd x k),   s = self + 8 hops,
// which runs as real MFMA tiles on the split real / imaginary parts:
//     C_re += M_re X_re - M_im X_im,   C_im += M_re X_im + M_im X_re.
// Workgroup = one site; wave w owns rows [16w, 16w+16) of C (nd <= 64).  The
// k right-hand-side columns of every X_s are staged once in LDS (one coalesced
// pass per RHS), so each block entry is read once for all right-hand sides.
// The FP32 form uses v_mfma_f32_16x16x4_f32 on FP32 blocks; the FP16-storage
// form uses v_mfma_f32_16x16x16_f16 with the blocks as stored and X rounded to
// FP16 (FP32 accumulation in both).
//   16x16xK tile layout (lane l = 16 q + j):  A row j, k-slice q;  B column j,
//   k-slice q;  D column j, rows 4q .. 4q+3 in the four result registers.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

template <class S> struct MfmaK;
template <> struct MfmaK<float> { static constexpr int K = 4; };       // k per instruction, FP32 inputs
template <> struct MfmaK<_Float16> { static constexpr int K = 16; };   // k per instruction, FP16 inputs

__device__ __forceinline__ f32x4 mma(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma(f16x4 a, f16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// columns of X staged in LDS for a batch of nr right-hand sides (the tile
// has 16): a batch of four needs a quarter of the LDS of sixteen, so more
// workgroups share a CU
__host__ __device__ __forceinline__ int mfma_cols(int nr) { return nr <= 4 ? 4 : (nr <= 8 ? 8 : 16); }

// A fragment of a column-major nd x nd block: row r, columns c0 .. c0+K/4-1
// of this lane's k-slice; zero outside the block.
template <class S>
__device__ __forceinline__ void a_frag(const cx<S>* __restrict__ A, int nd, int r, int c0, float sgn,
                                       typename std::conditional<std::is_same<S, float>::value, float, f16x4>::type& re,
                                       typename std::conditional<std::is_same<S, float>::value, float, f16x4>::type& im) {
    if constexpr (std::is_same<S, float>::value) {
        cx<float> a = (r < nd && c0 < nd) ? A[(size_t)c0 * nd + r] : czero<float>();
        re = sgn * a.re;
        im = sgn * a.im;
    } else {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int c = c0 + q;
            cx<_Float16> a = (r < nd && c < nd) ? A[(size_t)c * nd + r] : cx<_Float16>{_Float16(0), _Float16(0)};
            re[q] = sgn > 0 ? a.re : _Float16(-a.re);
            im[q] = sgn > 0 ? a.im : _Float16(-a.im);
        }
    }
}

// B fragment from the staged X [ndk][xs] (split re / im planes of type S):
// xs columns are staged (the batch rounded up to 4, 8 or 16); the lanes of
// the tile's other columns take zeros
template <class S>
__device__ __forceinline__ void b_frag(const S* __restrict__ Xre, const S* __restrict__ Xim, int c0, int j, int xs,
                                       typename std::conditional<std::is_same<S, float>::value, float, f16x4>::type& re,
                                       typename std::conditional<std::is_same<S, float>::value, float, f16x4>::type& im) {
    const bool on = j < xs;
    if constexpr (std::is_same<S, float>::value) {
        re = on ? Xre[c0 * xs + j] : 0.f;
        im = on ? Xim[c0 * xs + j] : 0.f;
    } else {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            re[q] = on ? Xre[(c0 + q) * xs + j] : _Float16(0);
            im[q] = on ? Xim[(c0 + q) * xs + j] : _Float16(0);
        }
    }
}

// C += A X over the ndk rows of X for one 16-row tile
template <class S>
__device__ __forceinline__ void tile_mma(const cx<S>* __restrict__ A, int nd, int ndk, int r, int lane, float sgn,
                                         const S* Xre, const S* Xim, int xs, f32x4& cre, f32x4& cim) {
    constexpr int K = MfmaK<S>::K;
    constexpr int KL = K / 4;   // k entries per lane
    const int q = lane >> 4, j = lane & 15;
    for (int k0 = 0; k0 < ndk; k0 += K) {
        const int c0 = k0 + q * KL;
        typename std::conditional<std::is_same<S, float>::value, float, f16x4>::type are, aim, bre, bim, naim;
        a_frag<S>(A, nd, r, c0, sgn, are, aim);
        b_frag<S>(Xre, Xim, c0, j, xs, bre, bim);
        naim = -aim;
        cre = mma(are, bre, cre);
        cre = mma(naim, bim, cre);
        cim = mma(are, bim, cim);
        cim = mma(aim, bre, cim);
    }
}

// The same for a compile-time padded extent NDK (the production nd = 40): all
// A fragments of the block are loaded before the first product, so a wave has
// NDK / K loads in flight instead of one per instruction step.
template <class S, int NDK>
__device__ __forceinline__ void tile_mma_fixed(const cx<S>* __restrict__ A, int nd, int r, int lane, float sgn,
                                               const S* Xre, const S* Xim, int xs, f32x4& cre, f32x4& cim) {
    constexpr int K = MfmaK<S>::K;
    constexpr int KL = K / 4;
    constexpr int NS = NDK / K;
    const int q = lane >> 4, j = lane & 15;
    typename std::conditional<std::is_same<S, float>::value, float, f16x4>::type are[NS], aim[NS];
#pragma unroll
    for (int t = 0; t < NS; t++) a_frag<S>(A, nd, r, t * K + q * KL, sgn, are[t], aim[t]);
#pragma unroll
    for (int t = 0; t < NS; t++) {
        typename std::conditional<std::is_same<S, float>::value, float, f16x4>::type bre, bim, naim;
        b_frag<S>(Xre, Xim, t * K + q * KL, j, xs, bre, bim);
        naim = -aim[t];
        cre = mma(are[t], bre, cre);
        cre = mma(naim, bim, cre);
        cim = mma(are[t], bim, cim);
        cim = mma(aim[t], bre, cim);
    }
}

// Fragments of one block for tile_mma_fixed, loaded ahead of their products
// so that the next block's loads overlap the current block's MFMA work.
template <class S, int NDK>
struct TileFrags {
    static constexpr int NS = NDK / MfmaK<S>::K;
    typename std::conditional<std::is_same<S, float>::value, float, f16x4>::type re[NS], im[NS];
};
template <class S, int NDK>
__device__ __forceinline__ void tile_load(const cx<S>* __restrict__ A, int nd, int r, int lane, float sgn,
                                          TileFrags<S, NDK>& f) {
    constexpr int K = MfmaK<S>::K, KL = K / 4;
    const int q = lane >> 4;
#pragma unroll
    for (int t = 0; t < TileFrags<S, NDK>::NS; t++) a_frag<S>(A, nd, r, t * K + q * KL, sgn, f.re[t], f.im[t]);
}
template <class S, int NDK>
__device__ __forceinline__ void tile_product(const TileFrags<S, NDK>& f, int lane, const S* Xre, const S* Xim, int xs,
                                             f32x4& cre, f32x4& cim) {
    constexpr int K = MfmaK<S>::K, KL = K / 4;
    const int q = lane >> 4, j = lane & 15;
#pragma unroll
    for (int t = 0; t < TileFrags<S, NDK>::NS; t++) {
        typename std::conditional<std::is_same<S, float>::value, float, f16x4>::type bre, bim, naim;
        b_frag<S>(Xre, Xim, t * K + q * KL, j, xs, bre, bim);
        naim = -f.im[t];
        cre = mma(f.re[t], bre, cre);
        cre = mma(naim, bim, cre);
        cim = mma(f.re[t], bim, cim);
        cim = mma(f.im[t], bre, cim);
    }
}

// the k x ndk tile product of one block: the unrolled form where the padded
// extent is the production one (NDK > 0), the loop otherwise
template <class S, int NDK>
__device__ __forceinline__ void tile_any(const cx<S>* __restrict__ A, int nd, int ndk, int r, int lane, float sgn,
                                         const S* Xre, const S* Xim, int xs, f32x4& cre, f32x4& cim) {
    if constexpr (NDK > 0) tile_mma_fixed<S, NDK>(A, nd, r, lane, sgn, Xre, Xim, xs, cre, cim);
    else tile_mma<S>(A, nd, ndk, r, lane, sgn, Xre, Xim, xs, cre, cim);
}

template <class S, int NDK = 0>
__global__ void __launch_bounds__(256) k_coarse_apply_mfma(CoarseOp<float, S> op, int par, int self_mode,
                                                           const cx<float>* __restrict__ in1, int hop_sign,
                                                           const cx<float>* in2, int post_inv, cx<float>* out, Mask mk,
                                                           long ld, int nr) {
    constexpr int K = MfmaK<S>::K;
    extern __shared__ char smem_raw[];
    __shared__ const cx<S>* mat[9];
    __shared__ const cx<float>* vin[9];
    const Geom g = op.g;
    const int nd = op.nd;
    const int ndk = (nd + K - 1) / K * K;          // k extent padded to the instruction
    const int xs = mfma_cols(nr);                   // staged columns
    S* Xre = reinterpret_cast<S*>(smem_raw);        // [9][ndk][xs]
    S* Xim = Xre + 9 * ndk * xs;
    int p, i;
    if (par < 0) { p = blockIdx.x >= g.vh; i = blockIdx.x - p * g.vh; }
    else { p = par; i = blockIdx.x; }
    const size_t gs = (size_t)p * g.vh + i;
    const size_t nn = (size_t)nd * nd;
    const int t = threadIdx.x, nt = blockDim.x;
    // block and input of every slot: thread k < 8 finds neighbour k
    const int nself = (self_mode == CS_SELF || self_mode == CS_SELFINV) ? 1 : 0;
    if (t == 0 && nself) {
        mat[0] = (self_mode == CS_SELF) ? op.M + gs * 9 * nn : op.Minv + gs * nn;
        vin[0] = in1 + gs * nd;
    }
    if (hop_sign != 0 && t < 8) {
        int x[4];
        cb_coords(g, p, i, x);
        mat[nself + t] = op.M + (gs * 9 + 1 + t) * nn;
        vin[nself + t] = in2 + nb_global(g, p, x, t) * nd;
    }
    __syncthreads();
    const int ns = nself + (hop_sign != 0 ? 8 : 0);
    // stage X_s: entry (s, c, j), c fastest so each RHS column is read contiguously.
    // FP16 form: column j of every X_s is divided by sc[j], the largest modulus
    // of the column's reals over the 9 slots (a first pass over the inputs
    // finds it), so that the rounded inputs lie in [-1, 1] whatever the
    // vector's magnitude; the products are scaled back in FP32.
    constexpr bool F16 = std::is_same<S, _Float16>::value;
    __shared__ float sc[16];
    if constexpr (F16) {
        if (t < 16) sc[t] = 0.f;
        __syncthreads();
        for (int e = t; e < ns * xs * ndk; e += nt) {
            const int sl = e / (xs * ndk), rem = e - sl * xs * ndk;
            const int j = rem / ndk, c = rem - j * ndk;
            if (c < nd && j < nr && mk.on(j)) {
                const cx<float> v = vin[sl][(size_t)j * ld + c];
                const float m = fmaxf(fabsf(v.re), fabsf(v.im));
                if (m > 0.f) atomicMax(reinterpret_cast<int*>(sc) + j, __float_as_int(m));
            }
        }
        __syncthreads();
        for (int e = t; e < ns * xs * ndk; e += nt) {
            const int sl = e / (xs * ndk), rem = e - sl * xs * ndk;
            const int j = rem / ndk, c = rem - j * ndk;
            cx<float> v = czero<float>();
            if (c < nd && j < nr && mk.on(j)) v = vin[sl][(size_t)j * ld + c];
            const float inv = sc[j] > 0.f ? 1.f / sc[j] : 0.f;
            Xre[(sl * ndk + c) * xs + j] = S(v.re * inv);
            Xim[(sl * ndk + c) * xs + j] = S(v.im * inv);
        }
    } else {
        for (int e = t; e < ns * xs * ndk; e += nt) {
            const int sl = e / (xs * ndk), rem = e - sl * xs * ndk;
            const int j = rem / ndk, c = rem - j * ndk;
            cx<float> v = czero<float>();
            if (c < nd && j < nr && mk.on(j)) v = vin[sl][(size_t)j * ld + c];
            Xre[(sl * ndk + c) * xs + j] = S(v.re);
            Xim[(sl * ndk + c) * xs + j] = S(v.im);
        }
    }
    __syncthreads();
    const int w = t >> 6, lane = t & 63;
    const int ntile = (nd + 15) / 16;
    const int r = 16 * w + (lane & 15);
    f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
    if (w < ntile) {
        auto sgn_of = [&](int sl) { return (sl >= nself && hop_sign < 0) ? -1.f : 1.f; };
        if constexpr (NDK > 0) {
            // software pipeline over the slots: block sl + 1 loads while block sl multiplies
            TileFrags<S, NDK> fa, fb;
            tile_load<S, NDK>(mat[0], nd, r, lane, sgn_of(0), fa);
            for (int sl = 0; sl < ns; sl += 2) {
                if (sl + 1 < ns) tile_load<S, NDK>(mat[sl + 1], nd, r, lane, sgn_of(sl + 1), fb);
                tile_product<S, NDK>(fa, lane, Xre + sl * ndk * xs, Xim + sl * ndk * xs, xs, cre, cim);
                if (sl + 1 >= ns) break;
                if (sl + 2 < ns) tile_load<S, NDK>(mat[sl + 2], nd, r, lane, sgn_of(sl + 2), fa);
                tile_product<S, NDK>(fb, lane, Xre + (sl + 1) * ndk * xs, Xim + (sl + 1) * ndk * xs, xs, cre, cim);
            }
        } else {
            for (int sl = 0; sl < ns; sl++)
                tile_mma<S>(mat[sl], nd, ndk, r, lane, sgn_of(sl), Xre + sl * ndk * xs, Xim + sl * ndk * xs, xs, cre, cim);
        }
    }
    // result rows 16w + 4q + v, column j
    const int q = lane >> 4, j = lane & 15;
    const bool jon = j < nr && mk.on(j);
    if constexpr (F16) {
#pragma unroll
        for (int v = 0; v < 4; v++) {
            cre[v] *= sc[j];
            cim[v] *= sc[j];
        }
    }
    if (self_mode == CS_IDENT && w < ntile && jon) {
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int row = 16 * w + 4 * q + v;
            if (row < nd) {
                cx<float> a = in1[(size_t)j * ld + gs * nd + row];
                cre[v] += a.re;
                cim[v] += a.im;
            }
        }
    }
    if (!post_inv) {
        if (w < ntile && jon) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int row = 16 * w + 4 * q + v;
                if (row < nd) out[(size_t)j * ld + gs * nd + row] = cx<float>{cre[v], cim[v]};
            }
        }
        return;
    }
    // post multiplication by the self-block inverse: stage the result as a new X
    // (FP16 form: scaled per column as above)
    __syncthreads();
    for (int e = t; e < ndk * xs; e += nt) {   // clear (padding rows stay zero)
        Xre[e] = S(0.f);
        Xim[e] = S(0.f);
    }
    if constexpr (F16) {
        if (t < 16) sc[t] = 0.f;
        __syncthreads();
        if (w < ntile) {
            float m = 0.f;
#pragma unroll
            for (int v = 0; v < 4; v++)
                if (16 * w + 4 * q + v < nd) m = fmaxf(m, fmaxf(fabsf(cre[v]), fabsf(cim[v])));
            if (m > 0.f) atomicMax(reinterpret_cast<int*>(sc) + j, __float_as_int(m));
        }
    }
    __syncthreads();
    float inv = 1.f;
    if constexpr (F16) inv = sc[j] > 0.f ? 1.f / sc[j] : 0.f;
    if (w < ntile) {
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int row = 16 * w + 4 * q + v;
            if (row < nd && j < xs) {
                Xre[row * xs + j] = S(cre[v] * inv);
                Xim[row * xs + j] = S(cim[v] * inv);
            }
        }
    }
    __syncthreads();
    if (w < ntile) {
        f32x4 dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
        tile_any<S, NDK>(op.Minv + gs * nn, nd, ndk, r, lane, 1.f, Xre, Xim, xs, dre, dim);
        if constexpr (F16) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                dre[v] *= sc[j];
                dim[v] *= sc[j];
            }
        }
        if (jon) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int row = 16 * w + 4 * q + v;
                if (row < nd) out[(size_t)j * ld + gs * nd + row] = cx<float>{dre[v], dim[v]};
            }
        }
    }
}

template <class S>
static size_t mfma_lds_bytes(int nd, int nr) {
    const int K = MfmaK<S>::K;
    const int ndk = (nd + K - 1) / K * K;
    return 2 * sizeof(S) * 9 * (size_t)ndk * mfma_cols(nr);
}

// ---------------------------------------------------------------------------
// The same stencil split by rows: workgroup = (site, chunk of RC rows) with RC
// rows of a block column making one 128-byte line, so a small coarse lattice
// still spreads over every CU.  Lane (rl, cg) of a wavefront accumulates row
// rl of the chunk over the columns q = cg, cg + CG, ... of the site's panel
// (self block, then the 8 hop blocks, or the 8 folded blocks B_k); the column
// groups meet through lane shuffles and the wavefronts in LDS.  No post
// multiplication: the folded blocks carry the self inverse where it is needed.
// ---------------------------------------------------------------------------
template <class T, class S, int RC>
__global__ void __launch_bounds__(256) k_coarse_rows(CoarseOp<T, S> op, int par, int self_mode,
                                                     const cx<T>* __restrict__ in1, int hop_sign, int fold,
                                                     const cx<T>* in2, cx<T>* out, Mask mk, long ld, InScale isc) {
    constexpr int CG = 64 / RC;          // column groups per wavefront
    constexpr int PF = (CG >= 4) ? 12 * (8 / CG) : 24;   // block entries a lane loads at once
    if (!mk.on(blockIdx.y)) return;
    {
        const long off = blockIdx.y * ld;
        if (in1) in1 += off;
        if (in2) in2 += off;
        out += off;
    }
    __shared__ cx<T> X[9 * 64];          // staged inputs [slot][nd] (nd <= 64), hop sign folded in
    __shared__ cx<T> part[4][RC];
    __shared__ const cx<T>* vin[9];
    const Geom g = op.g;
    const int nd = op.nd;
    const int nrc = (nd + RC - 1) / RC;
    const int site = blockIdx.x / nrc, rc = blockIdx.x - site * nrc;
    int p, i;
    if (par < 0) { p = site >= g.vh; i = site - p * g.vh; }
    else { p = par; i = site; }
    const size_t gs = (size_t)p * g.vh + i;
    const size_t nn = (size_t)nd * nd;
    const int nself = (self_mode == CS_SELF) ? 1 : 0;
    const cx<S>* panel = fold ? op.B + (size_t)i * 8 * nn : op.M + (gs * 9 + 1 - nself) * nn;
    // input vectors of the panel's column slots: thread k < 8 finds neighbour k
    if (threadIdx.x == 0 && nself) vin[0] = in1 + gs * nd;
    if (hop_sign != 0 && threadIdx.x < 8) {
        int x[4];
        cb_coords(g, p, i, x);
        vin[nself + threadIdx.x] = in2 + nb_global(g, p, x, threadIdx.x) * nd;
    }
    const int ns = nself + (hop_sign != 0 ? 8 : 0);
    const int Q = ns * nd;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
    const int rl = lane % RC, cg = lane / RC;
    const int row = rc * RC + rl;
    const bool rok = row < nd;
    const int qs = w * CG + cg, qstep = nw * CG;
    const cx<S>* A = panel + (rok ? row : 0);
    cx<S> a[PF];
    auto load = [&](int qb) {
#pragma unroll
        for (int u = 0; u < PF; u++) {
            const int q = qb + u * qstep;
            a[u] = (rok && q < Q) ? A[(size_t)q * nd] : cx<S>{S(0), S(0)};
        }
    };
    load(qs);   // in flight while the inputs are staged
    // factors of the two inputs (stored GMRES basis vectors carry theirs in the state)
    T f1 = T(1), f2 = T(1);
    if (isc.st) {
        const T f = T(isc.st[blockIdx.y].sc[isc.j]);
        if (isc.which & 1) f1 = f;
        if (isc.which & 2) f2 = f;
    }
    if (hop_sign < 0) f2 = -f2;
    __syncthreads();
    for (int e = t; e < Q; e += blockDim.x) {
        const int s2 = e / nd;
        const cx<T> v = vin[s2][e - s2 * nd];
        X[e] = ((s2 >= nself) ? f2 : f1) * v;
    }
    __syncthreads();
    cx<T> acc = czero<T>();
    for (int qb = qs; qb < Q; qb += PF * qstep) {
        if (qb != qs) load(qb);
#pragma unroll
        for (int u = 0; u < PF; u++) {
            const int q = qb + u * qstep;
            if (q < Q) acc += ccast<T>(a[u]) * X[q];
        }
    }
#pragma unroll
    for (int o = RC; o < 64; o <<= 1) {
        acc.re += __shfl_xor(acc.re, o, 64);
        acc.im += __shfl_xor(acc.im, o, 64);
    }
    if (cg == 0) part[w][rl] = acc;
    __syncthreads();
    if (w == 0 && cg == 0 && rok) {
        cx<T> tot = (self_mode == CS_IDENT) ? f1 * in1[gs * nd + row] : czero<T>();
        for (int q = 0; q < nw; q++) tot += part[q][rl];
        out[gs * nd + row] = tot;
    }
}

template <class T, class S>
static void launch_rows(const CoarseOp<T, S>& op, int par, int self_mode, const cx<T>* in1, int hop_sign, int fold,
                        const cx<T>* in2, cx<T>* out, hipStream_t s, Mask mk, int nr, long ld, InScale isc) {
    constexpr int RC = 128 / (int)sizeof(cx<S>);   // rows per 128-byte line
    const int nsite = (par < 0) ? 2 * op.g.vh : op.g.vh;
    const int nrc = (op.nd + RC - 1) / RC;
    dim3 grid(nsite * nrc, nr);
    k_coarse_rows<T, S, RC><<<grid, 256, 0, s>>>(op, par, self_mode, in1, hop_sign, fold, in2, out, mk, ld, isc);
}

// B_k(x) = Minv(x) M_{1+k}(x): workgroup (even site i, hop k), FP64 sums
template <class T>
__global__ void k_coarse_fold(int nd, const cx<T>* __restrict__ M, const cx<T>* __restrict__ Minv,
                              cx<T>* __restrict__ B) {
    const int i = blockIdx.x, k = blockIdx.y;
    const size_t nn = (size_t)nd * nd;
    const cx<T>* Mi = Minv + (size_t)i * nn;
    const cx<T>* Mk = M + ((size_t)i * 9 + 1 + k) * nn;
    cx<T>* Bk = B + ((size_t)i * 8 + k) * nn;
    for (int e = threadIdx.x; e < (int)nn; e += blockDim.x) {
        const int c = e / nd, r = e - c * nd;   // column-major entry (r, c)
        cx<double> s = czero<double>();
        for (int q = 0; q < nd; q++) s += ccast<double>(Mi[(size_t)q * nd + r]) * ccast<double>(Mk[(size_t)c * nd + q]);
        Bk[e] = ccast<T>(s);
    }
}

template <class T>
void coarse_fold_inverse(const Geom& g, int nd, const cx<T>* M, const cx<T>* Minv, cx<T>* B, hipStream_t s) {
    dim3 grid(g.vh, 8);
    k_coarse_fold<T><<<grid, 256, 0, s>>>(nd, M, Minv, B);
}

template <class T, class S>
bool coarse_uses_mfma(const CoarseOp<T, S>& op, int nr) {
    return std::is_same<T, float>::value && op.mfma && nr >= 2 && nr <= 16 && op.nd <= 64;
}

template <class T, class S>
void coarse_apply_folded(const CoarseOp<T, S>& op, const cx<T>* in1, int hop_sign, const cx<T>* in2, cx<T>* out,
                         hipStream_t s, Mask mk, int nr, long ld, InScale isc) {
    if (!op.B || op.nd > 64) throw std::invalid_argument("coarse_apply_folded: no folded blocks on this level");
    launch_rows(op, 0, in1 ? CS_IDENT : CS_NONE, in1, hop_sign, 1, in2, out, s, mk, nr, ld, isc);
}

template <class T, class S>
void coarse_apply(const CoarseOp<T, S>& op, int par, int self_mode, const cx<T>* in1, int hop_sign, const cx<T>* in2,
                  bool post_inv, cx<T>* out, hipStream_t s, Mask mk, int nr, long ld, InScale isc) {
    const bool rows = !post_inv && self_mode != CS_SELFINV && op.nd <= 64;
    if (isc.st && (coarse_uses_mfma(op, nr) || !rows))
        throw std::invalid_argument("coarse_apply: scaled inputs need the row-split vector-unit form");
    int nsite = (par < 0) ? 2 * op.g.vh : op.g.vh;
    if constexpr (std::is_same<T, float>::value) {
        // the matrix-core form serves FP32 arithmetic with 2..16 right-hand sides and nd <= 64
        if (op.mfma && nr >= 2 && nr <= 16 && op.nd <= 64) {
            constexpr int K = MfmaK<S>::K;
            constexpr int NDK40 = (40 + K - 1) / K * K;
            if (op.nd == 40)
                k_coarse_apply_mfma<S, NDK40><<<nsite, 64 * 3, mfma_lds_bytes<S>(op.nd, nr), s>>>(
                    op, par, self_mode, in1, hop_sign, in2, post_inv ? 1 : 0, out, mk, ld, nr);
            else
                k_coarse_apply_mfma<S><<<nsite, 64 * ((op.nd + 15) / 16), mfma_lds_bytes<S>(op.nd, nr), s>>>(
                    op, par, self_mode, in1, hop_sign, in2, post_inv ? 1 : 0, out, mk, ld, nr);
            return;
        }
    }
    // without the post multiplication by the inverse the row-split form applies
    if (rows) {
        launch_rows(op, par, self_mode, in1, hop_sign, 0, in2, out, s, mk, nr, ld, isc);
        return;
    }
    // the vector-unit kernel reads the site's blocks as one panel: the self
    // inverse is not stored next to the hop blocks
    if (self_mode == CS_SELFINV && hop_sign != 0)
        throw std::invalid_argument("coarse_apply: the self-block inverse combines with no hop term");
    int nslot = ((self_mode == CS_SELF || self_mode == CS_SELFINV) ? 1 : 0) + (hop_sign != 0 ? 8 : 0);
    // at most one prefetch batch of (block, column) pairs per wavefront where the
    // workgroup size allows
    int nw = std::max(1, std::min(CA_WAVES, (nslot * op.nd + CaPre<S>::N - 1) / CaPre<S>::N));
    if (post_inv) nw = std::max(nw, std::min(CA_WAVES, (op.nd + CaPre<S>::INV - 1) / CaPre<S>::INV));
    dim3 grid(nsite, nr);
    k_coarse_apply<T, S><<<grid, 64 * nw, 0, s>>>(op, par, self_mode, in1, hop_sign, in2, post_inv ? 1 : 0, out, mk, ld);
}

// ---------------------------------------------------------------------------
// Persistent coarsest-level GMRES cycle (one cooperative launch).
//
// On small coarse lattices every Arnoldi step of the odd-even GMRES is a
// handful of tiny launches whose latency dominates.  This kernel runs all the
// steps of one restart cycle, for every RHS of the batch, inside one launch of
// G co-resident workgroups that meet at grid barriers:
//   A  t_e = A_ee^{-1} D_eo v_j          (even sites, spread over workgroups)
//   B  w   = A_oo v_j - D_oe t_e          (odd sites)
//   C  partial inner products V_i^H w    (odd entries cut into G chunks)
//   D  h = sum of the partials (fixed order, in every workgroup), w -= V h,
//      partial ||w||^2
//   E  ||w||, Givens update of the Hessenberg column (identical arithmetic
//      in every workgroup; workgroup 0 writes the GmDev state), w /= ||w||
// Each step is five barriers; the stop test is the device GMRES's own.  The
// barrier is a counter/generation pair updated with device-scope atomics; a
// wait that exceeds its spin limit raises `abort` and every workgroup leaves,
// so the kernel always drains.
// ---------------------------------------------------------------------------
static constexpr int COOP_NT = 256;
static constexpr int COOP_MAXR = 16;

__device__ __forceinline__ bool coop_barrier(unsigned* bar, int* abort_flag, unsigned nblk) {
    __syncthreads();
    __shared__ int ok_s;
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        const unsigned g = __hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblk - 1) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(bar + 1, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
                if (++spins > (1L << 24)) {   // about a second: give up rather than hang
                    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        __threadfence();
        ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0;
}

// out(site) = [post Minv] ( self(x) in1 + hop_sign sum_k M_k in2(x_k) ) for one
// site with the workgroup's 4 wavefronts (lane r owns row r; nd <= 64)
template <class T, class S>
__device__ __forceinline__ void coop_site_apply(const CoarseOp<T, S>& op, int p, int i, int self_mode,
                                                const cx<T>* in1, int hop_sign, const cx<T>* in2, bool post_inv,
                                                cx<T>* out, cx<T> (*part)[64], cx<T>* buf, const cx<S>** mat,
                                                const cx<T>** vin) {
    const Geom& g = op.g;
    const int nd = op.nd;
    const int t = threadIdx.x, w = t >> 6, r = t & 63;
    const size_t gs = (size_t)p * g.vh + i;
    const size_t nn = (size_t)nd * nd;
    const int nself = (self_mode == CS_SELF || self_mode == CS_SELFINV) ? 1 : 0;
    const int ns = nself + (hop_sign != 0 ? 8 : 0);
    if (t < ns) {
        if (t < nself) {
            mat[0] = (self_mode == CS_SELF) ? op.M + gs * 9 * nn : op.Minv + gs * nn;
            vin[0] = in1 + gs * nd;
        } else {
            const int k = t - nself;
            int x[4], y[4];
            cb_coords(g, p, i, x);
            nb_coords(g, x, k, y);
            mat[t] = op.M + (gs * 9 + 1 + k) * nn;
            vin[t] = in2 + ((size_t)(1 - p) * g.vh + cb_index(g, y)) * nd;
        }
    }
    __syncthreads();
    const int Q = ns * nd, per = (Q + 3) / 4;
    const int q0 = w * per, q1 = min(Q, q0 + per);
    cx<T> acc = czero<T>();
    if (r < nd) {
        int q = q0;
        while (q < q1) {
            const int sl = q / nd, c0 = q - sl * nd, c1 = min(nd, c0 + (q1 - q));
            const cx<S>* A = mat[sl] + r;
            const cx<T>* v = vin[sl];
            cx<T> a2 = czero<T>();
            for (int c = c0; c < c1; c++) a2 += ccast<T>(A[(size_t)c * nd]) * v[c];
            if (sl >= nself && hop_sign < 0) acc -= a2;
            else acc += a2;
            q += c1 - c0;
        }
    }
    part[w][r] = acc;
    __syncthreads();
    cx<T> tot = czero<T>();
    if (w == 0 && r < nd) {
        tot = (self_mode == CS_IDENT) ? in1[gs * nd + r] : czero<T>();
        for (int q = 0; q < 4; q++) tot += part[q][r];
    }
    if (!post_inv) {
        if (w == 0 && r < nd) out[gs * nd + r] = tot;
        __syncthreads();
        return;
    }
    if (w == 0) buf[r] = tot;
    __syncthreads();
    const int per2 = (nd + 3) / 4, c0 = w * per2, c1 = min(nd, c0 + per2);
    cx<T> a3 = czero<T>();
    if (r < nd) {
        const cx<S>* A = op.Minv + gs * nn + r;
        for (int c = c0; c < c1; c++) a3 += ccast<T>(A[(size_t)c * nd]) * buf[c];
    }
    part[w][r] = a3;
    __syncthreads();
    if (w == 0 && r < nd) {
        cx<T> s2 = czero<T>();
        for (int q = 0; q < 4; q++) s2 += part[q][r];
        out[gs * nd + r] = s2;
    }
    __syncthreads();
}

// sum of v over the workgroup (COOP_NT threads), returned to every thread
__device__ __forceinline__ double coop_sum(double v, double* sh) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0;
    for (int q = 0; q < COOP_NT / 64; q++) s += sh[q];
    return s;
}

__device__ __forceinline__ cx<double> cdivd(cx<double> a, cx<double> b) {
    double d = norm2(b);
    return cx<double>{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

template <class T, class S>
__global__ void __launch_bounds__(COOP_NT) k_gmres_coop(CoarseOp<T, S> op, cx<T>* __restrict__ V, long ldv, long nfull,
                                                        cx<T>* tmp, GmDev* st, int nr, int m, cx<double>* part,
                                                        unsigned* bar, int* abort_flag) {
    __shared__ cx<T> ap_part[4][64];
    __shared__ cx<T> ap_buf[64];
    __shared__ const cx<S>* ap_mat[9];
    __shared__ const cx<T>* ap_vin[9];
    __shared__ double sh[COOP_NT / 64];
    __shared__ cx<double> cs_s[COOP_MAXR][32], sn_s[COOP_MAXR][32], g_s[COOP_MAXR][33], h_s[COOP_MAXR][33];
    __shared__ cx<double> col_s[COOP_MAXR][34];
    __shared__ int stop_s[COOP_MAXR], its_s[COOP_MAXR], fixed_s[COOP_MAXR], maxit_s[COOP_MAXR];
    __shared__ double tol_s[COOP_MAXR], hn_s[COOP_MAXR];
    const unsigned G = gridDim.x;
    const int wg = blockIdx.x, t = threadIdx.x;
    const int vh = op.g.vh;
    const long nh = (long)vh * op.nd;
    // private copy of the rotation state (every workgroup updates it identically)
    int j0 = 0;
    for (int r = 0; r < nr; r++) {
        const GmDev* sr = st + r;
        if (t < 32) { cs_s[r][t] = sr->cs[t]; sn_s[r][t] = sr->sn[t]; }
        if (t < 33) g_s[r][t] = sr->g[t];
        if (t == 0) {
            stop_s[r] = sr->stop;
            its_s[r] = sr->its;
            fixed_s[r] = sr->fixed;
            maxit_s[r] = sr->maxit;
            tol_s[r] = sr->tol_abs;
        }
        if (!sr->stop) j0 = sr->j;   // the running RHS share j
    }
    __syncthreads();
    const long chunk = (nh + G - 1) / G;
    const long e0 = min(nh, (long)wg * chunk), e1 = min(nh, e0 + chunk);
    for (int j = j0; j < m; j++) {
        int live = 0;
        for (int r = 0; r < nr; r++) live += !stop_s[r];
        if (!live) break;
        // A: t_e = A_ee^{-1} D_eo v_j (odd part of v_j)
        for (int s = wg; s < vh; s += G)
            for (int r = 0; r < nr; r++) {
                if (stop_s[r]) continue;
                const cx<T>* vj = V + (size_t)j * ldv + (size_t)r * nfull;
                coop_site_apply(op, 0, s, CS_NONE, (const cx<T>*)nullptr, 1, vj, true, tmp + (size_t)r * nfull,
                                ap_part, ap_buf, ap_mat, ap_vin);
            }
        if (!coop_barrier(bar, abort_flag, G)) return;
        // B: w = A_oo v_j - D_oe t_e, written as v_{j+1}
        for (int s = wg; s < vh; s += G)
            for (int r = 0; r < nr; r++) {
                if (stop_s[r]) continue;
                const cx<T>* vj = V + (size_t)j * ldv + (size_t)r * nfull;
                coop_site_apply(op, 1, s, CS_SELF, vj, -1, tmp + (size_t)r * nfull, false,
                                V + (size_t)(j + 1) * ldv + (size_t)r * nfull, ap_part, ap_buf, ap_mat, ap_vin);
            }
        if (!coop_barrier(bar, abort_flag, G)) return;
        // C: partial inner products over this workgroup's chunk of the odd entries
        for (int r = 0; r < nr; r++) {
            if (stop_s[r]) continue;
            const cx<T>* Vr = V + (size_t)r * nfull + nh;
            const cx<T>* w = Vr + (size_t)(j + 1) * ldv;
            for (int i = 0; i <= j; i++) {
                double re = 0, im = 0;
                for (long e = e0 + t; e < e1; e += COOP_NT) {
                    cx<T> a = Vr[(size_t)i * ldv + e], b = w[e];
                    re += (double)a.re * b.re + (double)a.im * b.im;
                    im += (double)a.re * b.im - (double)a.im * b.re;
                }
                re = coop_sum(re, sh);
                im = coop_sum(im, sh);
                if (t == 0) part[((size_t)r * 34 + i) * G + wg] = cx<double>{re, im};
            }
        }
        if (!coop_barrier(bar, abort_flag, G)) return;
        // D: h (fixed-order sum of the partials), w -= V h, partial ||w||^2
        for (int r = 0; r < nr; r++) {
            if (stop_s[r]) continue;
            for (int i = t; i <= j; i += COOP_NT) {
                cx<double> hsum = czero<double>();
                for (unsigned q = 0; q < G; q++) hsum += part[((size_t)r * 34 + i) * G + q];
                h_s[r][i] = hsum;
            }
        }
        __syncthreads();
        for (int r = 0; r < nr; r++) {
            if (stop_s[r]) continue;
            const cx<T>* Vr = V + (size_t)r * nfull + nh;
            cx<T>* w = V + (size_t)(j + 1) * ldv + (size_t)r * nfull + nh;
            double acc = 0;
            for (long e = e0 + t; e < e1; e += COOP_NT) {
                cx<T> we = w[e];
                for (int i = 0; i <= j; i++) we -= ccast<T>(h_s[r][i]) * Vr[(size_t)i * ldv + e];
                w[e] = we;
                acc += (double)norm2(we);
            }
            acc = coop_sum(acc, sh);
            if (t == 0) part[((size_t)r * 34 + 33) * G + wg] = cx<double>{acc, 0.0};
        }
        if (!coop_barrier(bar, abort_flag, G)) return;
        // E: ||w||, Givens update (same arithmetic as the step-by-step kernels), scale
        if (t < nr && !stop_s[t]) {
            const int r = t;
            double n2 = 0;
            for (unsigned q = 0; q < G; q++) n2 += part[((size_t)r * 34 + 33) * G + q].re;
            const double hn = sqrt(n2);
            cx<double>* col = col_s[r];
            for (int i = 0; i <= j; i++) col[i] = h_s[r][i];
            col[j + 1] = cx<double>{hn, 0.0};
            for (int i = 0; i < j; i++) {
                cx<double> a = col[i], b = col[i + 1];
                col[i] = conj(cs_s[r][i]) * a + conj(sn_s[r][i]) * b;
                col[i + 1] = -(sn_s[r][i] * a) + cs_s[r][i] * b;
            }
            cx<double> a = col[j], b = col[j + 1];
            const double den = sqrt(norm2(a) + norm2(b));
            if (den == 0.0) { cs_s[r][j] = cx<double>{1.0, 0.0}; sn_s[r][j] = czero<double>(); }
            else { cs_s[r][j] = cx<double>{a.re / den, a.im / den}; sn_s[r][j] = cx<double>{b.re / den, b.im / den}; }
            col[j] = conj(cs_s[r][j]) * a + conj(sn_s[r][j]) * b;
            col[j + 1] = czero<double>();
            g_s[r][j + 1] = -(sn_s[r][j] * g_s[r][j]);
            g_s[r][j] = conj(cs_s[r][j]) * g_s[r][j];
            its_s[r] += 1;
            const double resid = sqrt(norm2(g_s[r][j + 1]));
            int stop = (fixed_s[r] > 0) ? (its_s[r] >= fixed_s[r]) : ((resid <= tol_s[r]) || (its_s[r] >= maxit_s[r]));
            if (hn == 0.0) stop = 1;
            hn_s[r] = hn;
            if (wg == 0) {
                GmDev* sr = st + r;
                for (int i = 0; i <= j + 1; i++) sr->H[(size_t)j * 33 + i] = col[i];
                sr->cs[j] = cs_s[r][j];
                sr->sn[j] = sn_s[r][j];
                sr->g[j] = g_s[r][j];
                sr->g[j + 1] = g_s[r][j + 1];
                sr->its = its_s[r];
                sr->j = j + 1;
                sr->stop = stop;
                sr->scale = (hn > 0) ? 1.0 / hn : 0.0;
                sr->sc[j + 1] = 1.0;   // this kernel stores its basis vectors normalised
            }
            stop_s[r] = stop;
        }
        __syncthreads();
        for (int r = 0; r < nr; r++) {
            if (stop_s[r]) continue;   // (a RHS that stopped in this step is not scaled, as before)
            cx<T>* w = V + (size_t)(j + 1) * ldv + (size_t)r * nfull + nh;
            const T sc = T(1.0 / hn_s[r]);
            for (long e = e0 + t; e < e1; e += COOP_NT) w[e] = sc * w[e];
        }
        if (!coop_barrier(bar, abort_flag, G)) return;
    }
}

// Largest grid the cooperative launch admits (0 when not supported)
template <class T, class S>
int coarse_gmres_coop_max_grid() {
    int dev = 0, ncu = 0, per = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_gmres_coop<T, S>, COOP_NT, 0) != hipSuccess)
        return 0;
    return per * ncu;
}

template <class T, class S>
hipError_t coarse_gmres_coop(const CoarseOp<T, S>& op, cx<T>* V, long ldv, long nfull, cx<T>* tmp, GmDev* st, int nr,
                             int m, cx<double>* part, unsigned* bar, int* abort_flag, int grid, hipStream_t s) {
    if (nr > COOP_MAXR || op.nd > 64 || m > 32 || grid < 1) return hipErrorInvalidValue;
    CoarseOp<T, S> a0 = op;
    void* args[] = {&a0, &V, &ldv, &nfull, &tmp, &st, &nr, &m, &part, &bar, &abort_flag};
    return hipLaunchCooperativeKernel((const void*)k_gmres_coop<T, S>, dim3(grid), dim3(COOP_NT), args, 0, s);
}

// ---------------------------------------------------------------------------
// self-block inverse: Gauss-Jordan with partial pivoting on [A | I] in FP64
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_coarse_selfinv(Geom g, int nd, const cx<T>* __restrict__ M, cx<T>* __restrict__ Minv, int* bad) {
    extern __shared__ char smem_raw[];
    cx<double>* a = reinterpret_cast<cx<double>*>(smem_raw);  // row-major [nd][2nd]
    __shared__ int piv;
    __shared__ double pmax[1024 / 64];
    __shared__ int pidx[1024 / 64];
    const size_t gs = blockIdx.x;
    const size_t nn = (size_t)nd * nd;
    const int t = threadIdx.x, nt = blockDim.x, w2 = 2 * nd;
    for (int e = t; e < nd * w2; e += nt) {
        int r = e / w2, c = e % w2;
        a[e] = (c < nd) ? ccast<double>(M[gs * 9 * nn + (size_t)c * nd + r]) : ((c - nd == r) ? cx<double>{1.0, 0.0} : czero<double>());
    }
    __syncthreads();
    int singular = 0;
    for (int c = 0; c < nd; c++) {
        // pivot search over rows c..nd-1
        double best = -1.0;
        int bi = c;
        for (int r = c + t; r < nd; r += nt) {
            double v = norm2(a[r * w2 + c]);
            if (v > best) { best = v; bi = r; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            double ob = __shfl_xor(best, o, 64);
            int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if ((t & 63) == 0) { pmax[t >> 6] = best; pidx[t >> 6] = bi; }
        __syncthreads();
        if (t == 0) {
            double b = pmax[0];
            int bidx = pidx[0];
            for (int q = 1; q < (nt + 63) / 64; q++)
                if (pmax[q] > b || (pmax[q] == b && pidx[q] < bidx)) { b = pmax[q]; bidx = pidx[q]; }
            piv = (b > 0.0) ? bidx : -1;
        }
        __syncthreads();
        int pr = piv;
        if (pr < 0) { singular = 1; break; }
        if (pr != c)
            for (int j = t; j < w2; j += nt) {
                cx<double> tmp = a[c * w2 + j]; a[c * w2 + j] = a[pr * w2 + j]; a[pr * w2 + j] = tmp;
            }
        __syncthreads();
        cx<double> pv = a[c * w2 + c];
        double d = norm2(pv);
        cx<double> ip = {pv.re / d, -pv.im / d};
        __syncthreads();
        for (int j = t; j < w2; j += nt) a[c * w2 + j] = a[c * w2 + j] * ip;
        __syncthreads();
        for (int e = t; e < nd * w2; e += nt) {
            int r = e / w2, j = e % w2;
            if (r == c) continue;
            cx<double> f = a[r * w2 + c];
            if (j == c) continue;
            a[e] -= f * a[c * w2 + j];
        }
        __syncthreads();
        for (int r = t; r < nd; r += nt)
            if (r != c) a[r * w2 + c] = czero<double>();
        __syncthreads();
    }
    if (singular) {
        if (t == 0) atomicAdd(bad, 1);
        return;
    }
    for (int e = t; e < (int)nn; e += nt) {
        int c = e / nd, r = e % nd;  // column-major output
        Minv[gs * nn + e] = ccast<T>(a[r * w2 + nd + c]);
    }
}

template <class T>
void coarse_self_inverse(const Geom& g, int nd, const cx<T>* M, cx<T>* Minv, int* bad, hipStream_t s) {
    size_t lds = sizeof(cx<double>) * nd * 2 * nd;
    k_coarse_selfinv<T><<<2 * g.vh, 256, lds, s>>>(g, nd, M, Minv, bad);
}

// ---------------------------------------------------------------------------
// layout conversion of coarse vectors and blocks
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_coarse_import(Geom g, int nd, int n, const double* __restrict__ canon, cx<T>* __restrict__ out) {
    long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long vol = 2L * g.vh;
    if (e >= vol * nd) return;
    long s = e / nd;
    int c = (int)(e % nd);
    int x[4];
    canon_coords(g.d, s, x);
    size_t gs = lay_global(g, x);
    const cx<double>* src = reinterpret_cast<const cx<double>*>(canon);
    for (int v = 0; v < n; v++) out[(size_t)v * vol * nd + gs * nd + c] = ccast<T>(src[(size_t)v * vol * nd + s * nd + c]);
}

template <class T>
__global__ void k_coarse_export(Geom g, int nd, int n, const cx<T>* __restrict__ in, double* __restrict__ canon) {
    long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long vol = 2L * g.vh;
    if (e >= vol * nd) return;
    long s = e / nd;
    int c = (int)(e % nd);
    int x[4];
    canon_coords(g.d, s, x);
    size_t gs = lay_global(g, x);
    cx<double>* dst = reinterpret_cast<cx<double>*>(canon);
    for (int v = 0; v < n; v++) dst[(size_t)v * vol * nd + s * nd + c] = ccast<double>(in[(size_t)v * vol * nd + gs * nd + c]);
}

// blocks: layout [site][nslot][nd][nd] column-major -> canonical [site][nslot][nd][nd] row-major
template <class T>
__global__ void k_coarse_export_blocks(Geom g, int nd, int nslot, const cx<T>* __restrict__ in, double* __restrict__ canon) {
    long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long vol = 2L * g.vh;
    long nn = (long)nd * nd;
    if (e >= vol * nslot * nn) return;
    long s = e / (nslot * nn);
    long rem = e % (nslot * nn);
    int slot = (int)(rem / nn);
    int q = (int)(rem % nn);
    int r = q / nd, c = q % nd;
    int x[4];
    canon_coords(g.d, s, x);
    size_t gs = lay_global(g, x);
    cx<double>* dst = reinterpret_cast<cx<double>*>(canon);
    dst[e] = ccast<double>(in[(gs * nslot + slot) * nn + (size_t)c * nd + r]);
}

template <class T>
__global__ void k_coarse_shift(Geom g, int nd, double dm, cx<T>* M) {
    long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (e >= 2L * g.vh * nd) return;
    long s = e / nd;
    int r = (int)(e % nd);
    M[(s * 9) * nd * nd + (size_t)r * nd + r].re += T(dm);
}

template <class T>
void coarse_import_vector(const Geom& g, int nd, int n, const double* canon, cx<T>* out, hipStream_t s) {
    long tot = 2L * g.vh * nd;
    k_coarse_import<T><<<nblk_of(tot, 256), 256, 0, s>>>(g, nd, n, canon, out);
}
template <class T>
void coarse_export_vector(const Geom& g, int nd, int n, const cx<T>* in, double* canon, hipStream_t s) {
    long tot = 2L * g.vh * nd;
    k_coarse_export<T><<<nblk_of(tot, 256), 256, 0, s>>>(g, nd, n, in, canon);
}
template <class T>
void coarse_export_blocks(const Geom& g, int nd, int nslot, const cx<T>* in, double* canon, hipStream_t s) {
    long tot = 2L * g.vh * nslot * nd * nd;
    k_coarse_export_blocks<T><<<nblk_of(tot, 256), 256, 0, s>>>(g, nd, nslot, in, canon);
}
template <class T>
void coarse_shift_diag(const Geom& g, int nd, double dm, cx<T>* M, hipStream_t s) {
    long tot = 2L * g.vh * nd;
    k_coarse_shift<T><<<nblk_of(tot, 256), 256, 0, s>>>(g, nd, dm, M);
}

// ---------------------------------------------------------------------------
// coarse SAP half sweep (same algebra as the fine kernel, dense site blocks):
// workgroup = one block, thread = (local site l, row r) for both parities.
// ---------------------------------------------------------------------------
// row r of a column-major block times v; block entries and v are loaded in
// batches of RA_BATCH (many loads in flight, the sum still in column order)
// (a 4-byte complex -- FP16 storage -- is loaded as one 32-bit word and
// converted after the batch: converting each half as it arrives would make the
// compiler wait for every load in turn)
template <class S>
using cx_word = typename std::conditional<sizeof(cx<S>) == 4, unsigned int, cx<S>>::type;

template <class T, class S, int RA_BATCH>
__device__ __forceinline__ cx<T> row_apply(const cx<S>* __restrict__ A, int nd, int r, const cx<T>* v) {
    using W = cx_word<S>;
    const W* Aw = reinterpret_cast<const W*>(A);
    cx<T> s = czero<T>();
    for (int c0 = 0; c0 < nd; c0 += RA_BATCH) {
        W a[RA_BATCH];
        cx<T> x[RA_BATCH];
#pragma unroll
        for (int u = 0; u < RA_BATCH; u++) {
            const bool in = c0 + u < nd;
            a[u] = in ? Aw[(size_t)(c0 + u) * nd + r] : W{};
            x[u] = in ? v[c0 + u] : czero<T>();
        }
#pragma unroll
        for (int u = 0; u < RA_BATCH; u++)
            if (c0 + u < nd) s += ccast<T>(__builtin_bit_cast(cx<S>, a[u])) * x[u];
    }
    return s;
}

// One right-hand side per workgroup (grid.y = RHS).
// NTMAX: the workgroup size the kernel is compiled for (wider batches of
// loads where fewer threads leave more registers per thread)
template <class T, class S, int NTMAX>
__global__ void __launch_bounds__(NTMAX) k_coarse_sap1(CoarseOp<T, S> op, const int* __restrict__ blocks, const cx<T>* __restrict__ b,
                             cx<T>* __restrict__ z, int mr_steps, long ld, Mask mk) {
    if (!mk.on(blockIdx.y)) return;
    b += blockIdx.y * ld;
    z += blockIdx.y * ld;
    extern __shared__ char smem_raw[];
    const Geom g = op.g;
    const int nd = op.nd, bvh = g.bvh;
    const size_t nn = (size_t)nd * nd;
    constexpr int RB = NTMAX <= 512 ? 20 : 8;
    cx<T>* so = reinterpret_cast<cx<T>*>(smem_raw);  // [bvh][nd] odd-site field
    cx<T>* se = so + bvh * nd;                        // even-site field
    cx<T>* tm = se + bvh * nd;                        // temporary (even)
    double* red = reinterpret_cast<double*>(tm + bvh * nd);
    const int blk = blocks[blockIdx.x];
    const int base = blk << g.lbvh;
    const int t = threadIdx.x;
    const bool act = t < bvh * nd;
    const int l = act ? t / nd : 0, r = act ? t % nd : 0;
    const int i = base + l;
    int xe[4], xo[4], nbe[8], nbo[8];
    cb_coords(g, 0, i, xe);
    cb_coords(g, 1, i, xo);
    for (int k = 0; k < 8; k++) {
        int y[4];
        nb_coords(g, xe, k, y);
        nbe[k] = cb_index(g, y);
        nb_coords(g, xo, k, y);
        nbo[k] = cb_index(g, y);
    }
    const size_t ge = i, go = (size_t)g.vh + i;
    auto hop_glob = [&](size_t gs, int p, const int* nbj, const cx<T>* v) {
        cx<T> h = czero<T>();
        for (int k = 0; k < 8; k++) {
            size_t gy = (size_t)(1 - p) * g.vh + nbj[k];
            h += row_apply<T, S, RB>(op.M + (gs * 9 + 1 + k) * nn, nd, r, v + gy * nd);
        }
        return h;
    };
    auto hop_int = [&](size_t gs, const int* nbj, const cx<T>* buf) {
        cx<T> h = czero<T>();
        for (int k = 0; k < 8; k++) {
            if ((nbj[k] >> g.lbvh) != blk) continue;
            h += row_apply<T, S, RB>(op.M + (gs * 9 + 1 + k) * nn, nd, r, buf + (nbj[k] - base) * nd);
        }
        return h;
    };
    // t0_e = Minv (b_e - H z) - z_e
    cx<T> t0 = czero<T>(), rho = czero<T>(), eo = czero<T>(), sv = czero<T>();
    if (act) tm[l * nd + r] = b[ge * nd + r] - hop_glob(ge, 0, nbe, z);
    __syncthreads();
    if (act) {
        t0 = row_apply<T, S, RB>(op.Minv + ge * nn, nd, r, tm + l * nd) - z[ge * nd + r];
        se[l * nd + r] = t0;
        so[l * nd + r] = z[go * nd + r];
    }
    __syncthreads();
    // f_o = b_o - M0 z_o - H z - H_int t0
    if (act) rho = b[go * nd + r] - row_apply<T, S, RB>(op.M + go * 9 * nn, nd, r, so + l * nd) - hop_glob(go, 1, nbo, z) - hop_int(go, nbo, se);
    __syncthreads();
    if (act) so[l * nd + r] = rho;
    __syncthreads();
    const int lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
    for (int it = 0; it < mr_steps; it++) {
        if (act) tm[l * nd + r] = hop_int(ge, nbe, so);
        __syncthreads();
        cx<T> tv = czero<T>();
        if (act) tv = row_apply<T, S, RB>(op.Minv + ge * nn, nd, r, tm + l * nd);
        __syncthreads();
        if (act) se[l * nd + r] = tv;
        __syncthreads();
        double sr = 0, si = 0, ss = 0;
        if (act) {
            sv = row_apply<T, S, RB>(op.M + go * 9 * nn, nd, r, so + l * nd) - hop_int(go, nbo, se);
            cx<T> d = cmulc(sv, rho);
            sr = d.re; si = d.im; ss = norm2(sv);
        }
        sr = wave_sum(sr); si = wave_sum(si); ss = wave_sum(ss);
        if (lane == 0) { red[3 * w] = sr; red[3 * w + 1] = si; red[3 * w + 2] = ss; }
        __syncthreads();
        sr = si = ss = 0;
        for (int q = 0; q < nw; q++) { sr += red[3 * q]; si += red[3 * q + 1]; ss += red[3 * q + 2]; }
        if (ss > 0 && act) {
            cx<T> alpha = {T(sr / ss), T(si / ss)};
            eo += alpha * rho;
            rho -= alpha * sv;
        }
        __syncthreads();
        if (act) so[l * nd + r] = (it + 1 < mr_steps) ? rho : eo;
        __syncthreads();
    }
    if (mr_steps == 0) {
        if (act) so[l * nd + r] = eo;
        __syncthreads();
    }
    if (act) tm[l * nd + r] = hop_int(ge, nbe, so);
    __syncthreads();
    if (act) {
        cx<T> ee = t0 - row_apply<T, S, RB>(op.Minv + ge * nn, nd, r, tm + l * nd);
        z[ge * nd + r] += ee;
        z[go * nd + r] += eo;
    }
}

// Coarse SAP half sweep on SAP blocks that are not the level's layout blocks
// (any extents with two colours, e.g. 2 x 3^3 on a 12 x 6^3 level): the block's
// sites come from tables (SapTab).  One workgroup per (block, RHS); thread
// (site l, row group rr) holds NR rows rr + q nd/NR of the even site l and the
// odd site l of the block (NR = 2 when bv * nd exceeds a workgroup).  Same
// algebra and summation order as k_coarse_sap1.
template <class T, class S, int NTMAX, int NR>
__global__ void __launch_bounds__(NTMAX) k_coarse_sap_t(CoarseOp<T, S> op, const int* __restrict__ blocks, SapTab tab,
                                                        const cx<T>* __restrict__ b, cx<T>* __restrict__ z,
                                                        int mr_steps, long ld, Mask mk) {
    if (!mk.on(blockIdx.y)) return;
    b += blockIdx.y * ld;
    z += blockIdx.y * ld;
    extern __shared__ char smem_raw[];
    const Geom g = op.g;
    const int nd = op.nd, bv = tab.bv, ndr = nd / NR;
    const size_t nn = (size_t)nd * nd;
    constexpr int RB = 8;
    cx<T>* so = reinterpret_cast<cx<T>*>(smem_raw);  // [bv][nd] odd-site field
    cx<T>* se = so + bv * nd;                         // even-site field
    cx<T>* tm = se + bv * nd;                         // temporary (even)
    double* red = reinterpret_cast<double*>(tm + bv * nd);
    const int blk = blocks[blockIdx.x];
    const int t = threadIdx.x;
    const bool act = t < bv * ndr;
    const int l = act ? t / ndr : 0, rr = act ? t % ndr : 0;
    const int ie = tab.sites[((size_t)blk * 2 + 0) * bv + l];
    const int io = tab.sites[((size_t)blk * 2 + 1) * bv + l];
    int xe[4], xo[4], nbe[8], nbo[8], lce[8], lco[8];
    cb_coords(g, 0, ie, xe);
    cb_coords(g, 1, io, xo);
    for (int k = 0; k < 8; k++) {
        int y[4];
        nb_coords(g, xe, k, y);
        nbe[k] = cb_index(g, y);
        size_t gy = (size_t)g.vh + nbe[k];
        lce[k] = (tab.of[gy] == blk) ? tab.loc[gy] : -1;
        nb_coords(g, xo, k, y);
        nbo[k] = cb_index(g, y);
        gy = (size_t)nbo[k];
        lco[k] = (tab.of[gy] == blk) ? tab.loc[gy] : -1;
    }
    const size_t ge = ie, go = (size_t)g.vh + io;
    auto hop_glob = [&](size_t gs, int p, const int* nbj, const cx<T>* v, int r) {
        cx<T> h = czero<T>();
        for (int k = 0; k < 8; k++) {
            size_t gy = (size_t)(1 - p) * g.vh + nbj[k];
            h += row_apply<T, S, RB>(op.M + (gs * 9 + 1 + k) * nn, nd, r, v + gy * nd);
        }
        return h;
    };
    auto hop_int = [&](size_t gs, const int* lcj, const cx<T>* buf, int r) {
        cx<T> h = czero<T>();
        for (int k = 0; k < 8; k++) {
            if (lcj[k] < 0) continue;
            h += row_apply<T, S, RB>(op.M + (gs * 9 + 1 + k) * nn, nd, r, buf + lcj[k] * nd);
        }
        return h;
    };
    cx<T> t0[NR], rho[NR], eo[NR], sv[NR];
#pragma unroll
    for (int q = 0; q < NR; q++) t0[q] = rho[q] = eo[q] = sv[q] = czero<T>();
    // t0_e = Minv (b_e - H z) - z_e
    if (act)
#pragma unroll
        for (int q = 0; q < NR; q++) {
            const int r = rr + q * ndr;
            tm[l * nd + r] = b[ge * nd + r] - hop_glob(ge, 0, nbe, z, r);
        }
    __syncthreads();
    if (act)
#pragma unroll
        for (int q = 0; q < NR; q++) {
            const int r = rr + q * ndr;
            t0[q] = row_apply<T, S, RB>(op.Minv + ge * nn, nd, r, tm + l * nd) - z[ge * nd + r];
            se[l * nd + r] = t0[q];
            so[l * nd + r] = z[go * nd + r];
        }
    __syncthreads();
    // f_o = b_o - M0 z_o - H z - H_int t0
    if (act)
#pragma unroll
        for (int q = 0; q < NR; q++) {
            const int r = rr + q * ndr;
            rho[q] = b[go * nd + r] - row_apply<T, S, RB>(op.M + go * 9 * nn, nd, r, so + l * nd) -
                     hop_glob(go, 1, nbo, z, r) - hop_int(go, lco, se, r);
        }
    __syncthreads();
    if (act)
#pragma unroll
        for (int q = 0; q < NR; q++) so[l * nd + rr + q * ndr] = rho[q];
    __syncthreads();
    const int lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
    for (int it = 0; it < mr_steps; it++) {
        if (act)
#pragma unroll
            for (int q = 0; q < NR; q++) {
                const int r = rr + q * ndr;
                tm[l * nd + r] = hop_int(ge, lce, so, r);
            }
        __syncthreads();
        cx<T> tv[NR];
#pragma unroll
        for (int q = 0; q < NR; q++) tv[q] = czero<T>();
        if (act)
#pragma unroll
            for (int q = 0; q < NR; q++) tv[q] = row_apply<T, S, RB>(op.Minv + ge * nn, nd, rr + q * ndr, tm + l * nd);
        __syncthreads();
        if (act)
#pragma unroll
            for (int q = 0; q < NR; q++) se[l * nd + rr + q * ndr] = tv[q];
        __syncthreads();
        double sr = 0, si = 0, ss = 0;
        if (act)
#pragma unroll
            for (int q = 0; q < NR; q++) {
                const int r = rr + q * ndr;
                sv[q] = row_apply<T, S, RB>(op.M + go * 9 * nn, nd, r, so + l * nd) - hop_int(go, lco, se, r);
                cx<T> d = cmulc(sv[q], rho[q]);
                sr += d.re; si += d.im; ss += norm2(sv[q]);
            }
        sr = wave_sum(sr); si = wave_sum(si); ss = wave_sum(ss);
        if (lane == 0) { red[3 * w] = sr; red[3 * w + 1] = si; red[3 * w + 2] = ss; }
        __syncthreads();
        sr = si = ss = 0;
        for (int v = 0; v < nw; v++) { sr += red[3 * v]; si += red[3 * v + 1]; ss += red[3 * v + 2]; }
        if (ss > 0 && act) {
            cx<T> alpha = {T(sr / ss), T(si / ss)};
#pragma unroll
            for (int q = 0; q < NR; q++) {
                eo[q] += alpha * rho[q];
                rho[q] -= alpha * sv[q];
            }
        }
        __syncthreads();
        if (act)
#pragma unroll
            for (int q = 0; q < NR; q++) so[l * nd + rr + q * ndr] = (it + 1 < mr_steps) ? rho[q] : eo[q];
        __syncthreads();
    }
    if (mr_steps == 0) {
        if (act)
#pragma unroll
            for (int q = 0; q < NR; q++) so[l * nd + rr + q * ndr] = eo[q];
        __syncthreads();
    }
    if (act)
#pragma unroll
        for (int q = 0; q < NR; q++) {
            const int r = rr + q * ndr;
            tm[l * nd + r] = hop_int(ge, lce, so, r);
        }
    __syncthreads();
    if (act)
#pragma unroll
        for (int q = 0; q < NR; q++) {
            const int r = rr + q * ndr;
            cx<T> ee = t0[q] - row_apply<T, S, RB>(op.Minv + ge * nn, nd, r, tm + l * nd);
            z[ge * nd + r] += ee;
            z[go * nd + r] += eo[q];
        }
}

// KR right-hand sides at once: every block entry loaded is applied to the KR
// vectors v + vo[q] (q < KR), accumulated into s[q] in the same column order
// as row_apply (so a RHS gets the same sums alone and in a group)
template <class T, class S, int KR, int RA_BATCH>
__device__ __forceinline__ void row_apply_k(const cx<S>* __restrict__ A, int nd, int r, const cx<T>* v,
                                            const size_t (&vo)[KR], cx<T> (&s)[KR]) {
    using W = cx_word<S>;
    const W* Aw = reinterpret_cast<const W*>(A);
#pragma unroll
    for (int q = 0; q < KR; q++) s[q] = czero<T>();
    for (int c0 = 0; c0 < nd; c0 += RA_BATCH) {
        W a[RA_BATCH];
#pragma unroll
        for (int u = 0; u < RA_BATCH; u++) a[u] = (c0 + u < nd) ? Aw[(size_t)(c0 + u) * nd + r] : W{};
#pragma unroll
        for (int q = 0; q < KR; q++) {
            cx<T> x[RA_BATCH];
#pragma unroll
            for (int u = 0; u < RA_BATCH; u++) x[u] = (c0 + u < nd) ? v[vo[q] + c0 + u] : czero<T>();
#pragma unroll
            for (int u = 0; u < RA_BATCH; u++)
                if (c0 + u < nd) s[q] += ccast<T>(__builtin_bit_cast(cx<S>, a[u])) * x[u];
        }
    }
}

// Coarse SAP half sweep for KR right-hand sides per workgroup: workgroup =
// (block, group of KR RHS), thread = (local site l, row r) for both parities;
// each block entry is loaded once per use for the whole group.  The fields of
// the group live in LDS as [q][bvh][nd].  Right-hand sides beyond nr or masked
// off take no part (their z is not touched).  NTMAX: the workgroup size the
// kernel is compiled for (wider batches of loads where fewer threads leave
// more registers per thread).
// Registers: the single-precision group of four is held to 128 VGPRs (four
// waves per SIMD, three workgroups of the 2^4 blocks per CU): t0 and e_o live
// in LDS and the column batches are shorter.  Latency, not bandwidth, bounds
// this kernel, and one workgroup per CU left most of the wait exposed.
template <class T, class S, int NTMAX, int KR>
__global__ void __launch_bounds__(NTMAX, (KR >= 4 && sizeof(T) == 4) ? 4 : 1) k_coarse_sap(CoarseOp<T, S> op, const int* __restrict__ blocks, const cx<T>* __restrict__ b,
                             cx<T>* __restrict__ z, int mr_steps, long ld, int nr, Mask mk) {
    const int q0 = blockIdx.y * KR;
    bool on[KR];
    bool any = false;
    size_t go_[KR], lo_[KR];   // offsets of member q in the global vector sets and in the LDS fields
#pragma unroll
    for (int q = 0; q < KR; q++) {
        on[q] = (q0 + q < nr) && mk.on(q0 + q);
        any |= on[q];
        // members past the batch read the first member's data (never written)
        go_[q] = (size_t)((q0 + q < nr) ? q : 0) * ld;
    }
    if (!any) return;
    b += (size_t)q0 * ld;
    z += (size_t)q0 * ld;
    extern __shared__ char smem_raw[];
    const Geom g = op.g;
    const int nd = op.nd, bvh = g.bvh;
    const size_t nn = (size_t)nd * nd;
    const size_t fs = (size_t)bvh * nd;               // one field of the block
#pragma unroll
    for (int q = 0; q < KR; q++) lo_[q] = q * fs;
    constexpr int RB = sizeof(T) == 8 ? (NTMAX <= 512 ? 4 : 2) : (NTMAX <= 512 && KR < 4 ? 10 : 5);
    cx<T>* so = reinterpret_cast<cx<T>*>(smem_raw);  // [KR][bvh][nd] odd-site fields
    cx<T>* se = so + KR * fs;                         // even-site fields
    cx<T>* tm = se + KR * fs;                         // temporaries (even)
    cx<T>* st = tm + KR * fs;                         // t0 (even), kept for the final update
    cx<T>* seo = st + KR * fs;                        // the odd-site correction e_o
    const int nw = (blockDim.x + 63) >> 6;
    double* red = reinterpret_cast<double*>(seo + KR * fs);  // [KR][nw][3]
    int* nbl = reinterpret_cast<int*>(red + 3 * KR * nw);   // [2][8][bvh] neighbour indices
    const int blk = blocks[blockIdx.x];
    const int base = blk << g.lbvh;
    const int t = threadIdx.x;
    const bool act = t < bvh * nd;
    const int l = act ? t / nd : 0, r = act ? t % nd : 0;
    const int i = base + l;
    if (act && r == 0) {
        int xe[4], xo[4];
        cb_coords(g, 0, i, xe);
        cb_coords(g, 1, i, xo);
        for (int k = 0; k < 8; k++) {
            int y[4];
            nb_coords(g, xe, k, y);
            nbl[k * bvh + l] = cb_index(g, y);
            nb_coords(g, xo, k, y);
            nbl[(8 + k) * bvh + l] = cb_index(g, y);
        }
    }
    // the neighbour indices of even (odd) sites: nbe[k * bvh] (nbo[k * bvh])
    const int* nbe = nbl + l;
    const int* nbo = nbl + 8 * bvh + l;
    __syncthreads();
    const size_t ge = i, go = (size_t)g.vh + i;
    // sum over the 8 hops of site gs (parity p) applied to the global vectors
    auto hop_glob = [&](size_t gs, int p, const int* nbj, cx<T> (&h)[KR]) {
#pragma unroll
        for (int q = 0; q < KR; q++) h[q] = czero<T>();
#pragma unroll 1
        for (int k = 0; k < 8; k++) {
            size_t gy = (size_t)(1 - p) * g.vh + nbj[k * bvh];
            cx<T> u[KR];
            row_apply_k<T, S, KR, RB>(op.M + (gs * 9 + 1 + k) * nn, nd, r, z + gy * nd, go_, u);
#pragma unroll
            for (int q = 0; q < KR; q++) h[q] += u[q];
        }
    };
    // sum over the hops that stay inside the block, applied to LDS fields
    auto hop_int = [&](size_t gs, const int* nbj, const cx<T>* buf, cx<T> (&h)[KR]) {
#pragma unroll
        for (int q = 0; q < KR; q++) h[q] = czero<T>();
#pragma unroll 1
        for (int k = 0; k < 8; k++) {
            const int j = nbj[k * bvh];
            if ((j >> g.lbvh) != blk) continue;
            cx<T> u[KR];
            row_apply_k<T, S, KR, RB>(op.M + (gs * 9 + 1 + k) * nn, nd, r, buf + (j - base) * nd, lo_, u);
#pragma unroll
            for (int q = 0; q < KR; q++) h[q] += u[q];
        }
    };
    const int me = l * nd + r;
    cx<T> rho[KR], sv[KR], h[KR], u[KR];
#pragma unroll
    for (int q = 0; q < KR; q++) {
        rho[q] = sv[q] = czero<T>();
        if (act) seo[q * fs + me] = czero<T>();
    }
    // t0_e = Minv (b_e - H z) - z_e
    if (act) {
        hop_glob(ge, 0, nbe, h);
#pragma unroll
        for (int q = 0; q < KR; q++) tm[q * fs + me] = b[go_[q] + ge * nd + r] - h[q];
    }
    __syncthreads();
    if (act) {
        row_apply_k<T, S, KR, RB>(op.Minv + ge * nn, nd, r, tm + l * nd, lo_, u);
#pragma unroll
        for (int q = 0; q < KR; q++) {
            const cx<T> t0 = u[q] - z[go_[q] + ge * nd + r];
            se[q * fs + me] = t0;
            st[q * fs + me] = t0;
            so[q * fs + me] = z[go_[q] + go * nd + r];
        }
    }
    __syncthreads();
    // f_o = b_o - M0 z_o - H z - H_int t0
    if (act) {
        cx<T> hg[KR], hi[KR];
        row_apply_k<T, S, KR, RB>(op.M + go * 9 * nn, nd, r, so + l * nd, lo_, u);
        hop_glob(go, 1, nbo, hg);
        hop_int(go, nbo, se, hi);
#pragma unroll
        for (int q = 0; q < KR; q++) rho[q] = b[go_[q] + go * nd + r] - u[q] - hg[q] - hi[q];
    }
    __syncthreads();
    if (act)
#pragma unroll
        for (int q = 0; q < KR; q++) so[q * fs + me] = rho[q];
    __syncthreads();
    const int lane = t & 63, w = t >> 6;
    for (int it = 0; it < mr_steps; it++) {
        if (act) {
            hop_int(ge, nbe, so, h);
#pragma unroll
            for (int q = 0; q < KR; q++) tm[q * fs + me] = h[q];
        }
        __syncthreads();
        if (act) row_apply_k<T, S, KR, RB>(op.Minv + ge * nn, nd, r, tm + l * nd, lo_, u);
        __syncthreads();
        if (act)
#pragma unroll
            for (int q = 0; q < KR; q++) se[q * fs + me] = u[q];
        __syncthreads();
        double sr[KR], si[KR], ss[KR];
        if (act) {
            row_apply_k<T, S, KR, RB>(op.M + go * 9 * nn, nd, r, so + l * nd, lo_, u);
            hop_int(go, nbo, se, h);
        }
#pragma unroll
        for (int q = 0; q < KR; q++) {
            sr[q] = si[q] = ss[q] = 0;
            if (act) {
                sv[q] = u[q] - h[q];
                cx<T> d = cmulc(sv[q], rho[q]);
                sr[q] = d.re; si[q] = d.im; ss[q] = norm2(sv[q]);
            }
            sr[q] = wave_sum(sr[q]); si[q] = wave_sum(si[q]); ss[q] = wave_sum(ss[q]);
            if (lane == 0) { red[(q * nw + w) * 3] = sr[q]; red[(q * nw + w) * 3 + 1] = si[q]; red[(q * nw + w) * 3 + 2] = ss[q]; }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < KR; q++) {
            double a0 = 0, a1 = 0, a2 = 0;
            for (int v = 0; v < nw; v++) { a0 += red[(q * nw + v) * 3]; a1 += red[(q * nw + v) * 3 + 1]; a2 += red[(q * nw + v) * 3 + 2]; }
            if (a2 > 0 && act) {
                cx<T> alpha = {T(a0 / a2), T(a1 / a2)};
                seo[q * fs + me] += alpha * rho[q];
                rho[q] -= alpha * sv[q];
            }
        }
        __syncthreads();
        if (act)
#pragma unroll
            for (int q = 0; q < KR; q++) so[q * fs + me] = (it + 1 < mr_steps) ? rho[q] : seo[q * fs + me];
        __syncthreads();
    }
    if (mr_steps == 0) {
        if (act)
#pragma unroll
            for (int q = 0; q < KR; q++) so[q * fs + me] = seo[q * fs + me];
        __syncthreads();
    }
    if (act) {
        hop_int(ge, nbe, so, h);
#pragma unroll
        for (int q = 0; q < KR; q++) tm[q * fs + me] = h[q];
    }
    __syncthreads();
    if (act) {
        row_apply_k<T, S, KR, RB>(op.Minv + ge * nn, nd, r, tm + l * nd, lo_, u);
#pragma unroll
        for (int q = 0; q < KR; q++) {
            if (!on[q]) continue;
            z[q * ld + ge * nd + r] += st[q * fs + me] - u[q];
            z[q * ld + go * nd + r] += seo[q * fs + me];
        }
    }
}

// LDS of one member of a multi-RHS group: five block fields (odd sites, even
// sites, a temporary, t0, e_o) and the partial sums of three reductions per
// wave
template <class T>
static size_t coarse_sap_member_lds(int bvh, int nd) {
    const int nw = (bvh * nd + 63) / 64;
    return 5 * sizeof(cx<T>) * bvh * nd + 3 * sizeof(double) * nw;
}

template <class T, class S, int KR>
static void coarse_sap_launch(const CoarseOp<T, S>& op, const int* blocks, int nblocks, const cx<T>* b, cx<T>* z,
                              int mr_steps, hipStream_t s, int nr, long ld, Mask mk) {
    const int nt = ((op.g.bvh * op.nd + 63) / 64) * 64;
    if constexpr (KR == 1) {
        const size_t lds = 3 * sizeof(cx<T>) * op.g.bvh * op.nd + 3 * sizeof(double) * (nt / 64);
        dim3 grid(nblocks, nr);
        if (nt <= 512) k_coarse_sap1<T, S, 512><<<grid, nt, lds, s>>>(op, blocks, b, z, mr_steps, ld, mk);
        else k_coarse_sap1<T, S, 1024><<<grid, nt, lds, s>>>(op, blocks, b, z, mr_steps, ld, mk);
    } else {
        const size_t lds = coarse_sap_member_lds<T>(op.g.bvh, op.nd) * KR + 16 * sizeof(int) * op.g.bvh;
        dim3 grid(nblocks, (nr + KR - 1) / KR);
        if (nt <= 512) k_coarse_sap<T, S, 512, KR><<<grid, nt, lds, s>>>(op, blocks, b, z, mr_steps, ld, nr, mk);
        else k_coarse_sap<T, S, 1024, KR><<<grid, nt, lds, s>>>(op, blocks, b, z, mr_steps, ld, nr, mk);
    }
}

// Right-hand sides are taken in groups of four (two for a batch of two), so a
// block entry read from memory serves the whole group; a single RHS runs the
// one-RHS kernel.  Both compute the same sums in the same order.
template <class T, class S>
void coarse_sap_half(const CoarseOp<T, S>& op, const int* blocks, int nblocks, const cx<T>* b, cx<T>* z, int mr_steps,
                     hipStream_t s, int nr, long ld, Mask mk, SapTab tab) {
    if (nblocks <= 0) return;
    if (tab.bv > 0) {
        // SAP blocks from tables: one workgroup per (block, RHS)
        const int NR = (tab.bv * op.nd > 1024) ? 2 : 1;
        const int nt = ((tab.bv * op.nd / NR + 63) / 64) * 64;
        const size_t lds = 3 * sizeof(cx<T>) * tab.bv * op.nd + 3 * sizeof(double) * (nt / 64);
        dim3 grid(nblocks, nr);
        if (NR == 1) k_coarse_sap_t<T, S, 1024, 1><<<grid, nt, lds, s>>>(op, blocks, tab, b, z, mr_steps, ld, mk);
        else k_coarse_sap_t<T, S, 1024, 2><<<grid, nt, lds, s>>>(op, blocks, tab, b, z, mr_steps, ld, mk);
        return;
    }
    // LDS of a group: five block fields per member and the neighbour table
    // (kept within the 64 KB a workgroup gets without an opt-in)
    const size_t member = coarse_sap_member_lds<T>(op.g.bvh, op.nd), nbt = 16 * sizeof(int) * op.g.bvh;
    if (nr >= 3 && 4 * member + nbt <= 65536) coarse_sap_launch<T, S, 4>(op, blocks, nblocks, b, z, mr_steps, s, nr, ld, mk);
    else if (nr >= 2 && 2 * member + nbt <= 65536) coarse_sap_launch<T, S, 2>(op, blocks, nblocks, b, z, mr_steps, s, nr, ld, mk);
    else coarse_sap_launch<T, S, 1>(op, blocks, nblocks, b, z, mr_steps, s, nr, ld, mk);
}

// ---------------------------------------------------------------------------
// transfer between two coarse levels.  P columns: [N][vol_f][ndf] (layout
// order of the finer level); the coarser level has 2N unknowns per site.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void agg_site_c(const AggMap& m, const int xc[4], int s, int x[4]) {
    int l3 = s % m.a[3]; s /= m.a[3];
    int l2 = s % m.a[2]; s /= m.a[2];
    int l1 = s % m.a[1];
    int l0 = s / m.a[1];
    x[0] = xc[0] * m.a[0] + l0;
    x[1] = xc[1] * m.a[1] + l1;
    x[2] = xc[2] * m.a[2] + l2;
    x[3] = xc[3] * m.a[3] + l3;
}

// workgroup: coarser site; thread e < asz*ndf: (site s = e / ndf, row d = e % ndf)
template <class T, class S>
__global__ void k_coarse_restrict(AggMap m, int ndf, int N, const cx<S>* __restrict__ P, const cx<T>* __restrict__ in,
                                  cx<T>* __restrict__ out, long ldi, long ldo, Mask mk) {
    if (!mk.on(blockIdx.y)) return;
    in += blockIdx.y * ldi;
    out += blockIdx.y * ldo;
    extern __shared__ char smem_raw[];
    cx<double>* red = reinterpret_cast<cx<double>*>(smem_raw);
    const int gc = blockIdx.x;
    const int pc = gc >= m.c.vh, ic = gc - pc * m.c.vh;
    int xc[4];
    cb_coords(m.c, pc, ic, xc);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
    const long volf = 2L * m.f.vh;
    const int h0 = ndf / 2;
    const int ne = m.asz * ndf;
    // up to EPT entries per thread: their offsets, halves and input values are
    // found once for all N test vectors (the same sums in the same order)
    constexpr int EPT = 4;
    const bool held = ne <= EPT * (int)blockDim.x;
    size_t off[EPT];
    cx<T> vin[EPT];
    bool hi[EPT];
    if (held) {
#pragma unroll
        for (int u = 0; u < EPT; u++) {
            const int e = t + u * (int)blockDim.x;
            off[u] = 0;
            vin[u] = czero<T>();
            hi[u] = false;
            if (e < ne) {
                const int s = e / ndf, d = e % ndf;
                int x[4];
                agg_site_c(m, xc, s, x);
                off[u] = lay_global(m.f, x) * ndf + d;
                vin[u] = in[off[u]];
                hi[u] = d >= h0;
            }
        }
    }
    cx<double> acc[2];
    for (int k = 0; k < N; k++) {
        acc[0] = acc[1] = czero<double>();
        if (held) {
            const cx<S>* Pk = P + (size_t)k * volf * ndf;
#pragma unroll
            for (int u = 0; u < EPT; u++) {
                if (t + u * (int)blockDim.x >= ne) break;
                const cx<double> pr = ccast<double>(cmulc(ccast<T>(Pk[off[u]]), vin[u]));
                if (hi[u]) acc[1] += pr;
                else acc[0] += pr;
            }
        } else {
            for (int e = t; e < ne; e += blockDim.x) {
                int s = e / ndf, d = e % ndf;
                int x[4];
                agg_site_c(m, xc, s, x);
                size_t gf = lay_global(m.f, x);
                acc[d / h0] += ccast<double>(cmulc(ccast<T>(P[((size_t)k * volf + gf) * ndf + d]), in[gf * ndf + d]));
            }
        }
        for (int h = 0; h < 2; h++) {
            acc[h].re = wave_sum(acc[h].re);
            acc[h].im = wave_sum(acc[h].im);
            if (lane == 0) red[w * 2 * N + h * N + k] = acc[h];
        }
    }
    __syncthreads();
    for (int q = t; q < 2 * N; q += blockDim.x) {
        cx<double> s = czero<double>();
        for (int ww = 0; ww < nw; ww++) s += red[ww * 2 * N + q];
        out[(size_t)gc * 2 * N + q] = ccast<T>(s);
    }
}

template <class T, class S>
__global__ void k_coarse_prolong(AggMap m, int ndf, int N, const cx<S>* __restrict__ P, const cx<T>* __restrict__ in,
                                 cx<T>* __restrict__ out, long ldi, long ldo, Mask mk) {
    long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long volf = 2L * m.f.vh;
    if (e >= volf * ndf || !mk.on(blockIdx.y)) return;
    in += blockIdx.y * ldi;
    out += blockIdx.y * ldo;
    long gf = e / ndf;
    int d = (int)(e % ndf);
    int p = gf >= m.f.vh, i = (int)(gf - p * m.f.vh);
    int x[4], xc[4];
    cb_coords(m.f, p, i, x);
    for (int mu = 0; mu < 4; mu++) xc[mu] = x[mu] / m.a[mu];
    size_t gc = lay_global(m.c, xc);
    const int h = d / (ndf / 2);
    cx<T> s = czero<T>();
    for (int k = 0; k < N; k++) s += ccast<T>(P[((size_t)k * volf + gf) * ndf + d]) * in[gc * 2 * N + h * N + k];
    out[gf * ndf + d] = s;
}

template <class T, class S>
void coarse_restrict(const AggMap& m, int ndf, int N, const cx<S>* P, const cx<T>* in, cx<T>* out, hipStream_t s,
                     int nr, long ldi, long ldo, Mask mk) {
    int nt = 256;
    size_t lds = sizeof(cx<double>) * 2 * N * (nt / 64);
    dim3 grid(2 * m.c.vh, nr);
    k_coarse_restrict<T, S><<<grid, nt, lds, s>>>(m, ndf, N, P, in, out, ldi, ldo, mk);
}
template <class T, class S>
void coarse_prolong(const AggMap& m, int ndf, int N, const cx<S>* P, const cx<T>* in, cx<T>* out, hipStream_t s,
                    int nr, long ldi, long ldo, Mask mk) {
    long tot = 2L * m.f.vh * ndf;
    dim3 grid(nblk_of(tot, 256), nr);
    k_coarse_prolong<T, S><<<grid, 256, 0, s>>>(m, ndf, N, P, in, out, ldi, ldo, mk);
}

// modified Gram-Schmidt per (coarser site, half): rows = aggregate sites x ndf/2
template <class T>
__global__ void k_coarse_gs(AggMap m, int ndf, int N, const cx<T>* __restrict__ tv, cx<T>* __restrict__ P, int* bad) {
    __shared__ double red[2 * 16];
    const int gc = blockIdx.x, h = blockIdx.y;
    const int pc = gc >= m.c.vh, ic = gc - pc * m.c.vh;
    int xc[4];
    cb_coords(m.c, pc, ic, xc);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
    const int h0 = ndf / 2;
    const int rows = m.asz * h0;
    const bool act = t < rows;
    const long volf = 2L * m.f.vh;
    size_t off = 0;
    if (act) {
        int s = t / h0, d = h * h0 + t % h0;
        int x[4];
        agg_site_c(m, xc, s, x);
        size_t gf = lay_global(m.f, x);
        off = gf * ndf + d;
    }
    for (int k = 0; k < N; k++) {
        cx<double> q = act ? ccast<double>(tv[(size_t)k * volf * ndf + off]) : czero<double>();
        for (int j = 0; j < k; j++) {
            cx<double> pj = act ? ccast<double>(P[(size_t)j * volf * ndf + off]) : czero<double>();
            cx<double> d = cmulc(pj, q);
            d.re = wave_sum(d.re);
            d.im = wave_sum(d.im);
            __syncthreads();
            if (lane == 0) { red[2 * w] = d.re; red[2 * w + 1] = d.im; }
            __syncthreads();
            d = czero<double>();
            for (int ww = 0; ww < nw; ww++) { d.re += red[2 * ww]; d.im += red[2 * ww + 1]; }
            q -= d * pj;
        }
        double n2 = wave_sum(norm2(q));
        __syncthreads();
        if (lane == 0) red[2 * w] = n2;
        __syncthreads();
        n2 = 0;
        for (int ww = 0; ww < nw; ww++) n2 += red[2 * ww];
        double inv = 0;
        if (n2 > 0) inv = 1.0 / sqrt(n2);
        else if (t == 0) atomicAdd(bad, 1);
        if (act) P[(size_t)k * volf * ndf + off] = ccast<T>(inv * q);
    }
}

template <class T>
void coarse_gram_schmidt(const AggMap& m, int ndf, int N, const cx<T>* tv, cx<T>* P, int* bad, hipStream_t s) {
    int nt = ((m.asz * (ndf / 2) + 63) / 64) * 64;
    dim3 grid(2 * m.c.vh, 2);
    k_coarse_gs<T><<<grid, nt, 0, s>>>(m, ndf, N, tv, P, bad);
}

// next coarser operator from a coarse one: workgroup (coarser site, column b)
template <class T>
__global__ void k_coarse_assemble(CoarseOp<T> op, AggMap m, int N, const cx<T>* __restrict__ P, cx<T>* __restrict__ Mc) {
    extern __shared__ char smem_raw[];
    const int ndf = op.nd;
    const int h0 = ndf / 2;
    const size_t nnf = (size_t)ndf * ndf;
    cx<double>* red = reinterpret_cast<cx<double>*>(smem_raw);   // [nw][2N]
    const int gc = blockIdx.x, bcol = blockIdx.y;
    const int ndc = 2 * N, hb = bcol / N, kb = bcol % N;
    const int pc = gc >= m.c.vh, ic = gc - pc * m.c.vh;
    int xc[4];
    cb_coords(m.c, pc, ic, xc);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
    const bool act = t < m.asz * ndf;
    const long volf = 2L * m.f.vh;
    int s = act ? t / ndf : 0, r = act ? t % ndf : 0;
    int x[4];
    agg_site_c(m, xc, s, x);
    const int p = site_parity(x);
    const size_t gf = (size_t)p * m.f.vh + cb_index(m.f, x);
    // column b of P restricted to half hb, at site y
    auto pcol = [&](size_t gy, int c) -> cx<T> {
        return (c / h0 == hb) ? P[((size_t)kb * volf + gy) * ndf + c] : czero<T>();
    };
    for (int slot = 0; slot < 9; slot++) {
        cx<T> wv = czero<T>();
        if (act) {
            if (slot == 0) {
                for (int c = 0; c < ndf; c++) wv += op.M[(gf * 9) * nnf + (size_t)c * ndf + r] * pcol(gf, c);
                for (int k = 0; k < 8; k++) {
                    int y[4];
                    nb_coords(op.g, x, k, y);
                    if (y[0] / m.a[0] != xc[0] || y[1] / m.a[1] != xc[1] || y[2] / m.a[2] != xc[2] || y[3] / m.a[3] != xc[3]) continue;
                    size_t gy = (size_t)(1 - p) * m.f.vh + cb_index(m.f, y);
                    for (int c = 0; c < ndf; c++) wv += op.M[(gf * 9 + 1 + k) * nnf + (size_t)c * ndf + r] * pcol(gy, c);
                }
            } else {
                int k = slot - 1;
                int y[4];
                nb_coords(op.g, x, k, y);
                if (y[0] / m.a[0] != xc[0] || y[1] / m.a[1] != xc[1] || y[2] / m.a[2] != xc[2] || y[3] / m.a[3] != xc[3]) {
                    size_t gy = (size_t)(1 - p) * m.f.vh + cb_index(m.f, y);
                    for (int c = 0; c < ndf; c++) wv += op.M[(gf * 9 + 1 + k) * nnf + (size_t)c * ndf + r] * pcol(gy, c);
                }
            }
        }
        for (int a = 0; a < ndc; a++) {
            const int ha = a / N, ka = a % N;
            cx<double> d = czero<double>();
            if (act && r / h0 == ha) d = cmulc(ccast<double>(P[((size_t)ka * volf + gf) * ndf + r]), ccast<double>(wv));
            d.re = wave_sum(d.re);
            d.im = wave_sum(d.im);
            if (lane == 0) red[w * ndc + a] = d;
        }
        __syncthreads();
        for (int a = t; a < ndc; a += blockDim.x) {
            cx<double> sum = czero<double>();
            for (int ww = 0; ww < nw; ww++) sum += red[ww * ndc + a];
            Mc[(((size_t)gc * 9 + slot) * ndc + bcol) * ndc + a] = ccast<T>(sum);
        }
        __syncthreads();
    }
}

template <class T>
void coarse_assemble(const CoarseOp<T>& op, const AggMap& m, int N, const cx<T>* P, cx<T>* Mc, hipStream_t s) {
    int nt = ((m.asz * op.nd + 63) / 64) * 64;
    size_t lds = sizeof(cx<double>) * 2 * N * (nt / 64);
    dim3 grid(2 * m.c.vh, 2 * N);
    k_coarse_assemble<T><<<grid, nt, lds, s>>>(op, m, N, P, Mc);
}

// counter-based normal numbers (Philox4x32-10 + Box-Muller), element index site*nd + c
__device__ __forceinline__ void philox_c(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1; c[3] = (uint32_t)p0; c[0] = n0; c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

template <class T>
__global__ void k_coarse_random(Geom g, int nd, int n, unsigned long long seed, int sid, cx<T>* out) {
    long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long vol = 2L * g.vh;
    if (e >= vol * nd) return;
    long s = e / nd;
    int c = (int)(e % nd);
    int x[4];
    canon_coords(g.d, s, x);
    size_t gs = lay_global(g, x);
    for (int v = 0; v < n; v++) {
        unsigned long long el = (unsigned long long)e;
        uint32_t ctr[4] = {(uint32_t)el, (uint32_t)(el >> 32), (uint32_t)v, (uint32_t)sid};
        philox_c(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
        double u1 = (ctr[0] + 0.5) * (1.0 / 4294967296.0);
        double u2 = (ctr[1] + 0.5) * (1.0 / 4294967296.0);
        double rr = sqrt(-2.0 * log(u1));
        out[(size_t)v * vol * nd + gs * nd + c] = cx<T>{T(rr * cos(2.0 * M_PI * u2)), T(rr * sin(2.0 * M_PI * u2))};
    }
}

template <class T>
void coarse_random(const Geom& g, int nd, int n, unsigned long long seed, int sid, cx<T>* out, hipStream_t s) {
    long tot = 2L * g.vh * nd;
    k_coarse_random<T><<<nblk_of(tot, 256), 256, 0, s>>>(g, nd, n, seed, sid, out);
}

// operator kernels for compute type T and storage type S
#define DD_COARSE_OP_INST(T, S)                                                                                      \
    template int coarse_gmres_coop_max_grid<T, S>();                                                                 \
    template hipError_t coarse_gmres_coop<T, S>(const CoarseOp<T, S>&, cx<T>*, long, long, cx<T>*, GmDev*, int, int, \
                                                cx<double>*, unsigned*, int*, int, hipStream_t);                      \
    template void coarse_apply<T, S>(const CoarseOp<T, S>&, int, int, const cx<T>*, int, const cx<T>*, bool, cx<T>*,   \
                                     hipStream_t, Mask, int, long, InScale);                                        \
    template bool coarse_uses_mfma<T, S>(const CoarseOp<T, S>&, int);                                                \
    template void coarse_apply_folded<T, S>(const CoarseOp<T, S>&, const cx<T>*, int, const cx<T>*, cx<T>*,           \
                                            hipStream_t, Mask, int, long, InScale);                                 \
    template void coarse_sap_half<T, S>(const CoarseOp<T, S>&, const int*, int, const cx<T>*, cx<T>*, int, hipStream_t, \
                                        int, long, Mask, SapTab);                                                   \
    template void coarse_restrict<T, S>(const AggMap&, int, int, const cx<S>*, const cx<T>*, cx<T>*, hipStream_t, int, \
                                        long, long, Mask);                                                          \
    template void coarse_prolong<T, S>(const AggMap&, int, int, const cx<S>*, const cx<T>*, cx<T>*, hipStream_t, int,  \
                                       long, long, Mask);

#define DD_COARSE_INST(T)                                                                                                \
    DD_COARSE_OP_INST(T, T)                                                                                          \
    template void coarse_self_inverse<T>(const Geom&, int, const cx<T>*, cx<T>*, int*, hipStream_t);                  \
    template void coarse_fold_inverse<T>(const Geom&, int, const cx<T>*, const cx<T>*, cx<T>*, hipStream_t);          \
    template void coarse_import_vector<T>(const Geom&, int, int, const double*, cx<T>*, hipStream_t);                \
    template void coarse_export_vector<T>(const Geom&, int, int, const cx<T>*, double*, hipStream_t);                \
    template void coarse_export_blocks<T>(const Geom&, int, int, const cx<T>*, double*, hipStream_t);                \
    template void coarse_shift_diag<T>(const Geom&, int, double, cx<T>*, hipStream_t);                                \
    template void coarse_gram_schmidt<T>(const AggMap&, int, int, const cx<T>*, cx<T>*, int*, hipStream_t);          \
    template void coarse_assemble<T>(const CoarseOp<T>&, const AggMap&, int, const cx<T>*, cx<T>*, hipStream_t);     \
    template void coarse_random<T>(const Geom&, int, int, unsigned long long, int, cx<T>*, hipStream_t);

DD_COARSE_INST(double)
DD_COARSE_INST(float)
DD_COARSE_OP_INST(float, _Float16)

}  // namespace dd
