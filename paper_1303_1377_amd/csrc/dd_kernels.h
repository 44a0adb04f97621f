// dd_kernels.h -- host-side launchers of the HIP kernels (one translation unit
// per family: fine level, coarse levels, vector algebra).  All launchers are
// asynchronous on the given stream.
#pragma once
#include "dd_common.h"

namespace dd {

// Fine clover-Wilson operator in one precision, even-odd block-major layout.
//   U       [2][4][9][vh]  forward links of each site
//   clov    [2][72][vh]    packed A(x) = (m0+4) I + T(x), two Hermitian 6x6 blocks
//   clovinv [2][72][vh]    packed A(x)^{-1}
//   sched   SCHED_* flags: launch schedule of the stencil and SAP kernels
//           (results are identical for every choice; the autotuner picks one)
enum FineSched {
    SCHED_FUSED = 1,   // stencil: one workgroup covers both parities of its layout blocks
    SCHED_XCD = 2,     // stencil and SAP: XCD-contiguous workgroup order
    SCHED_LDS = 4,     // stencil: one workgroup per layout block staged in LDS
    SCHED_NO_MFMA = 8, // multi-RHS coarse stencil on the vector units instead of the matrix cores
    SCHED_GRAPH = 16,  // coarsest-level Arnoldi steps replayed as captured HIP graphs
    SCHED_COOP = 32,   // coarsest-level GMRES cycle as one persistent cooperative launch
    SCHED_COOP_ABORT = 64,  // test of the fallback: the cooperative cycle starts with its abort flag raised
};
// Fields are stored in S (T, or _Float16 for the FP16-storage preconditioner)
// and computed on in T.
template <class T, class S = T>
struct FineOp {
    Geom g;
    const cx<S>* U;
    const S* clov;
    const S* clovinv;
    int sched = SCHED_LDS | SCHED_XCD;
};

// Coarse stencil D_c on a level with nd unknowns per site.
//   M    [vol][9][nd][nd]  column-major blocks: slot 0 self, 1+mu couples x+mu,
//                          5+mu couples x-mu (layout site order)
//   Minv [vol][nd][nd]     column-major inverse of the self block
//   mfma  with 2..16 right-hand sides and FP32 arithmetic the apply runs on
//         the matrix cores (one launch for all RHS, each block entry read
//         once); 0: one workgroup per (site, RHS) on the vector units
//   B    [vh][8][nd][nd]   (coarsest level only, else null) the even sites' hop
//         blocks with the self inverse folded in, B_k(x) = Minv(x) M_{1+k}(x),
//         so that A_ee^{-1} D_eo needs no second pass over the site's result
template <class T, class S = T>
struct CoarseOp {
    Geom g;
    int nd;
    const cx<S>* M;
    const cx<S>* Minv;
    int mfma = 1;
    const cx<S>* B = nullptr;
};

// which right-hand sides of a batch a launch works on: flag r at p[r*stride];
// with invert = 1 a nonzero flag means "inactive" (e.g. a GMRES stop flag)
struct Mask {
    const int* p;
    int stride;
    int invert;
    __host__ __device__ __forceinline__ bool on(int r) const {
        return p == nullptr || ((p[(size_t)r * stride] != 0) != (invert != 0));
    }
};
static inline Mask all_rhs() { return Mask{nullptr, 1, 0}; }

// largest batch of right-hand sides, and per-RHS values passed by value
static constexpr int MAX_RHS = 16;
struct Coefs {
    double v[MAX_RHS];   // one real factor per right-hand side
};
struct Counts {
    int v[MAX_RHS];      // one count per right-hand side
};

// aggregation of a fine (or finer coarse) level onto the next coarser level
// SAP blocks of a coarse level that are not its layout blocks (bv > 0): for
// block B the layout indices of its even sites at sites[(2 B) bv ..] and of its
// odd sites at sites[(2 B + 1) bv ..] (bv of each); for every site (whole-layout
// index) its block in `of` and its position in its block's list in `loc`.
// bv = 0: the SAP blocks are the layout blocks.
struct SapTab {
    const int* sites = nullptr;
    const int* of = nullptr;
    const int* loc = nullptr;
    int bv = 0;
};

struct AggMap {
    Geom f;        // finer level layout
    Geom c;        // coarser level layout
    int a[4];      // aggregate lattice-block extents
    int asz;       // sites per aggregate
};

// ---- fine level (dd_fine.hip) ---------------------------------------------
template <class T> void fine_import_gauge(const Geom& g, const double* canon, cx<T>* U, hipStream_t s);
template <class T> void fine_import_spinor(const Geom& g, const double* canon, cx<T>* out, hipStream_t s);
template <class T> void fine_export_spinor(const Geom& g, const cx<T>* in, double* canon, hipStream_t s);
// clover from the FP64 layout links (four-leaf Q_{mu nu}), or from canonical
// user blocks T(x); writes packed A and A^{-1} in FP64.  `bad` counts singular blocks.
void fine_clover_from_links(const Geom& g, const cx<double>* U, double m0, double csw, double* clov,
                            double* clovinv, int* bad, hipStream_t s);
void fine_clover_from_user(const Geom& g, const double* canonT, double m0, double* clov, double* clovinv, int* bad,
                           hipStream_t s);
void fine_clover_shift(const Geom& g, double dm, double* clov, double* clovinv, int* bad, hipStream_t s);
void fine_clover_export(const Geom& g, const double* packed, double* canon, hipStream_t s);
// Batched launches: nr right-hand sides, vector r at base + r*ld (complex
// entries); RHS switched off by the mask are left untouched.
template <class T, class S>
void fine_dirac(const FineOp<T, S>& op, const cx<T>* in, cx<T>* out, hipStream_t s, int nr = 1, long ld = 0,
                Mask mk = all_rhs());
// the FP64 stencil applied to FP32 input vectors (converted as they are loaded)
void fine_dirac_from32(const FineOp<double>& op, const cx<float>* in, cx<double>* out, hipStream_t s, int nr = 1,
                       long ld = 0, Mask mk = all_rhs());
// one SAP half sweep: blocks listed in `blocks` (all of one colour); the block
// operator is loaded once and applied to every right-hand side of the batch
template <class T, class S>
void fine_sap_half(const FineOp<T, S>& op, const int* blocks, int nblocks, const cx<T>* b, cx<T>* z, int mr_steps,
                   hipStream_t s, int nr = 1, long ld = 0, Mask mk = all_rhs());
// LDS bytes one SAP workgroup needs for the layout blocks of g
template <class T> size_t fine_sap_lds_bytes(const Geom& g);
// P columns: [N][2][12][vh] (N fine spinors); coarse vectors: [cvol][2N] (layout order)
template <class T, class S>
void fine_restrict(const AggMap& m, int N, const cx<S>* P, const cx<T>* in, cx<T>* out, hipStream_t s, int nr = 1,
                   long ldi = 0, long ldo = 0, Mask mk = all_rhs());
template <class T, class S>
void fine_prolong(const AggMap& m, int N, const cx<S>* P, const cx<T>* in, cx<T>* out, hipStream_t s, int nr = 1,
                  long ldi = 0, long ldo = 0, Mask mk = all_rhs());
// the same three on FP16 spinor sets (hspin; offsets as for cx<T> sets)
template <class S>
void fine_sap_half_h(const FineOp<float, S>& op, const int* blocks, int nblocks, hspin b, hspin z, int mr_steps,
                     hipStream_t s, int nr, long ld, Mask mk);
template <class S>
void fine_restrict_h(const AggMap& m, int N, const cx<S>* P, hspin in, cx<float>* out, hipStream_t s, int nr, long ldi,
                     long ldo, Mask mk);
template <class S>
void fine_prolong_h(const AggMap& m, int N, const cx<S>* P, const cx<float>* in, hspin out, hipStream_t s, int nr,
                    long ldi, long ldo, Mask mk);
// FP16 spinor sets to and from FP64 / FP32 sets (nr vectors at stride ld) and
// x += sum_{j < m_r} y_r[j] Z_j for RHS r (Z_j of RHS r at Z + j ldz + r ldzr)
template <class S> void fine_hpack(int vh, const cx<S>* in, hspin out, long ld, int nr, Mask mk, hipStream_t s);
template <class D> void fine_hunpack(int vh, hspin in, cx<D>* out, long ld, int nr, Mask mk, hipStream_t s);
void fine_hlincomb(int vh, int m, hspin Z, long ldz, const cx<double>* y, cx<double>* x, hipStream_t s, int nr,
                   long ldzr, int ystride, long ldx, Mask mk, const Counts* per);
template <class T>
void fine_gram_schmidt(const AggMap& m, int N, const cx<T>* tv, cx<T>* P, int* bad, hipStream_t s);
template <class T>
void fine_assemble(const FineOp<T>& op, const AggMap& m, int N, const cx<T>* P, cx<T>* M, hipStream_t s);
template <class T> void fine_export_vectors(const Geom& g, int n, const cx<T>* in, double* canon, hipStream_t s);
// one parity p of the odd-even reduced operator:
//   out_p = M (sc * P self_p + cc * D_pq in_q),  P = A_pp if pre_a else I,
//   M = A_pp^{-1} if post_inv else I, D_pq the hopping term of D between the parities
template <class T, class S>
void fine_oe_hop(const FineOp<T, S>& op, int p, bool pre_a, bool post_inv, double sc, double cc, const cx<T>* self,
                 const cx<T>* in, cx<T>* out, hipStream_t s);
template <class T> void fine_import_vectors(const Geom& g, int n, const double* canon, cx<T>* out, hipStream_t s);
// draw n complex N(0,1) fine spinors from the counter-based generator
template <class T> void fine_random(const Geom& g, int n, unsigned long long seed, int stream_id, cx<T>* out, hipStream_t s);

// ---- coarse levels (dd_coarse.hip) ----------------------------------------
enum CoarseSelf { CS_NONE = 0, CS_IDENT = 1, CS_SELF = 2, CS_SELFINV = 3 };
// out(x) = [post Minv] ( self_mode(x) in1(x) + hop_sign * sum_k M_{1+k}(x) in2(x_k) )
// for the sites of parity `par` (0, 1) or all sites (par < 0).
// input scaling of the coarse stencil: the inputs flagged in `which` (1: in1,
// 2: in2) of right-hand side r are multiplied by st[r].sc[j] (GMRES basis
// vectors stored without their normalisation); vector-unit forms only
struct GmDev;
struct InScale {
    const GmDev* st = nullptr;
    int j = 0;
    int which = 0;
};
template <class T, class S>
void coarse_apply(const CoarseOp<T, S>& op, int par, int self_mode, const cx<T>* in1, int hop_sign, const cx<T>* in2,
                  bool post_inv, cx<T>* out, hipStream_t s, Mask mk = all_rhs(), int nr = 1, long ld = 0,
                  InScale isc = InScale{});
// whether coarse_apply takes the matrix-core form for nr right-hand sides
template <class T, class S>
bool coarse_uses_mfma(const CoarseOp<T, S>& op, int nr);
// out(x) = [in1(x)] + hop_sign * sum_k B_k(x) in2(x_k) on the even sites (op.B
// must be set; in1 may be null): A_ee^{-1} D_eo in one pass.  Not the
// matrix-core form: callers check coarse_uses_mfma first.
template <class T, class S>
void coarse_apply_folded(const CoarseOp<T, S>& op, const cx<T>* in1, int hop_sign, const cx<T>* in2, cx<T>* out,
                         hipStream_t s, Mask mk = all_rhs(), int nr = 1, long ld = 0, InScale isc = InScale{});
// B_k(x) = Minv(x) M_{1+k}(x) for the even sites x (FP64 accumulation)
template <class T>
void coarse_fold_inverse(const Geom& g, int nd, const cx<T>* M, const cx<T>* Minv, cx<T>* B, hipStream_t s);
// One restart cycle of the coarsest odd-even GMRES for nr <= 16 RHS in one
// cooperative launch of `grid` workgroups (see dd_coarse.hip); the GmDev states
// must have been started (gm_start) and v_0 normalised.  part: nr*34*grid
// complex doubles of scratch; bar: two zeroed words kept across launches;
// abort_flag: raised if a grid barrier wait exceeds its spin limit.
struct GmDev;
template <class T, class S> int coarse_gmres_coop_max_grid();
template <class T, class S>
hipError_t coarse_gmres_coop(const CoarseOp<T, S>& op, cx<T>* V, long ldv, long nfull, cx<T>* tmp, GmDev* st, int nr,
                             int m, cx<double>* part, unsigned* bar, int* abort_flag, int grid, hipStream_t s);
template <class T> void coarse_self_inverse(const Geom& g, int nd, const cx<T>* M, cx<T>* Minv, int* bad, hipStream_t s);
template <class T> void coarse_import_vector(const Geom& g, int nd, int n, const double* canon, cx<T>* out, hipStream_t s);
template <class T> void coarse_export_vector(const Geom& g, int nd, int n, const cx<T>* in, double* canon, hipStream_t s);
template <class T> void coarse_export_blocks(const Geom& g, int nd, int nslot, const cx<T>* in, double* canon, hipStream_t s);
template <class T> void coarse_shift_diag(const Geom& g, int nd, double dm, cx<T>* M, hipStream_t s);
template <class T, class S>
void coarse_sap_half(const CoarseOp<T, S>& op, const int* blocks, int nblocks, const cx<T>* b, cx<T>* z, int mr_steps,
                     hipStream_t s, int nr = 1, long ld = 0, Mask mk = all_rhs(), SapTab tab = SapTab{});
template <class T, class S>
void coarse_restrict(const AggMap& m, int ndf, int N, const cx<S>* P, const cx<T>* in, cx<T>* out, hipStream_t s,
                     int nr = 1, long ldi = 0, long ldo = 0, Mask mk = all_rhs());
template <class T, class S>
void coarse_prolong(const AggMap& m, int ndf, int N, const cx<S>* P, const cx<T>* in, cx<T>* out, hipStream_t s,
                    int nr = 1, long ldi = 0, long ldo = 0, Mask mk = all_rhs());
template <class T>
void coarse_gram_schmidt(const AggMap& m, int ndf, int N, const cx<T>* tv, cx<T>* P, int* bad, hipStream_t s);
template <class T>
void coarse_assemble(const CoarseOp<T>& op, const AggMap& m, int N, const cx<T>* P, cx<T>* Mc, hipStream_t s);
template <class T> void coarse_random(const Geom& g, int nd, int n, unsigned long long seed, int stream_id, cx<T>* out, hipStream_t s);

// ---- vector algebra (dd_blas.hip) -----------------------------------------
// lengths are in complex entries
template <class D, class S> void vec_convert(long n, const cx<S>* in, cx<D>* out, hipStream_t s);
template <class T> void vec_axpy(long n, cx<double> a, const cx<T>* x, cx<T>* y, hipStream_t s);   // y += a x
template <class T> void vec_xpay(long n, const cx<T>* x, cx<double> a, cx<T>* y, hipStream_t s);   // y = x + a y
template <class T> void vec_scale(long n, cx<double> a, cx<T>* x, hipStream_t s);
template <class T> void vec_sub(long n, const cx<T>* a, const cx<T>* b, cx<T>* out, hipStream_t s); // out = a - b
// out[i] = V_i^H w for i < m, V_i = V + i*ldv ; results in FP64 on the device.
// `work` must hold reduce_work_size(m) bytes; `count` is an int zeroed once.
size_t reduce_work_size(int m, int nr);
// Batch layout of the reductions: RHS r uses basis V + r*ldr, vector w + r*ldw
// and writes its results at out + r*ostride.
struct RedBatch {
    int nr;
    long ldr, ldw;
    int ostride;
    Mask mk;
};
static inline RedBatch single_rhs() { return RedBatch{1, 0, 0, 0, all_rhs()}; }
template <class T>
void vec_multidot(long n, int m, const cx<T>* V, long ldv, const cx<T>* w, cx<double>* out, void* work, int* count,
                  hipStream_t s, RedBatch rb = single_rhs());
// w -= sum_i h_i V_i (h in FP64 on the device, RHS r at h + r*ostride), then
// out[0].re = ||w||^2; with wc, the final w is also written in FP32 to
// wc + r*ldc (the input of a single-precision preconditioner)
template <class T>
void vec_update_norm(long n, int m, const cx<T>* V, long ldv, const cx<double>* h, cx<T>* w, cx<double>* out,
                     void* work, int* count, hipStream_t s, RedBatch rb = single_rhs(), const double* g = nullptr,
                     int gstride = 0, cx<float>* wc = nullptr, long ldc = 0);
// w -= sum_i h_i V_i and out_i = V_i^H w (the updated w) in one sweep over the
// basis: the first projection of a Gram-Schmidt pass and the inner products of
// its reorthogonalisation.  Returns false (nothing done) for m above its limit.
template <class T>
bool vec_update_dot(long n, int m, const cx<T>* V, long ldv, const cx<double>* h, cx<T>* w, cx<double>* out,
                    void* work, hipStream_t s, RedBatch rb = single_rhs(), const double* g = nullptr, int gstride = 0);
// g (may be NULL) scales the coefficients of the two updates: w -= sum_i g[r gstride + i] h_i V_i
// (basis vectors stored with factors, V_i = f_i stored_i, take g_i = f_i^2)
// g[r * gstride + idx] = c.v[r] for the RHS the mask keeps
void set_factor(double* g, int gstride, int idx, const Coefs& c, int nr, Mask mk, hipStream_t s);
// x += sum_i y_i Z_i (y in FP64 on the device; RHS r: Z + r*ldzr, y + r*ystride, x + r*ldx)
// over i < m, or i < per->v[r] when per-RHS counts are given
template <class T, class X>
void vec_lincomb(long n, int m, const cx<T>* Z, long ldz, const cx<double>* y, cx<X>* x, hipStream_t s, int nr = 1,
                 long ldzr = 0, int ystride = 0, long ldx = 0, Mask mk = all_rhs(), const Counts* per = nullptr);
template <class T>
void vec_finite_check(long n, const cx<T>* x, int* bad, hipStream_t s);

// batched element-wise operations: RHS r at base + r*ld, switched off by the mask
template <class D, class S>
void bvec_convert(long n, const cx<S>* in, cx<D>* out, long ld, int nr, Mask mk, hipStream_t s);
template <class T>
void bvec_sub(long n, const cx<T>* a, const cx<T>* b, cx<T>* out, long ld, int nr, Mask mk, hipStream_t s);
template <class T>
void bvec_scale(long n, const Coefs& c, cx<T>* x, long ld, int nr, Mask mk, hipStream_t s);
// d[r] = bit r of `bits` for r < n (device mask words written in stream order)
void set_flags(int* d, unsigned bits, int n, hipStream_t s);

// ---- device-resident GMRES(m) bookkeeping (coarsest level) -----------------
// The Hessenberg matrix, Givens rotations, residual estimate and stop flag of
// one restarted GMRES live on the device, so the host can enqueue several
// Arnoldi steps between synchronisations; every kernel of a step returns at
// once when `stop` is set.
struct alignas(16) GmDev {
    cx<double> H[33 * 32];   // rotated Hessenberg, column j at H[j*33 + i]
    cx<double> cs[32], sn[32], g[33], y[32];
    double sc[33];           // basis vector i = sc[i] * the stored vector i (stored
                             // vectors may be left unnormalised; 1 when normalised)
    double tol_abs;          // stop when |g_{j+1}| <= tol_abs
    double scale;            // 1/||w|| for the basis vector just produced
    int j;                   // columns completed in this cycle
    int its;                 // iterations in total
    int stop;                // converged, iteration cap or exact solution
    int m, maxit, fixed;
};
// One state per right-hand side: st[r]; reduction results of RHS r at
// res + r*rstride.  beta^2 from the norm reduction; first cycle also fixes tol_abs.
// A right-hand side the mask switches off is marked stopped with no columns;
// on a restart (first = 0) a stopped one keeps its iteration count and gets j = 0.
void gm_start(GmDev* st, const cx<double>* res, int rstride, double tol, int first, int m, int maxit, int fixed,
              int nr, hipStream_t s, Mask mk = all_rhs());
// out[3r..3r+2] = {j, its, stop} of st[r] (one small transfer reads a batch)
void gm_gather(const GmDev* st, int nr, int* out, hipStream_t s);
// y = R^{-1} g for the st->j columns of the cycle
void gm_solve(GmDev* st, int nr, hipStream_t s);
// x_r = st[r].scale * (src_r, or x_r itself when src is null) (skipped once
// st[r].stop unless ignore_stop)
template <class T>
void vec_scale_dev(long n, const GmDev* st, cx<T>* x, hipStream_t s, bool ignore_stop, int nr = 1, long ld = 0,
                   const cx<T>* src = nullptr);
// x_r += sum_{i < st[r].j} y_i sc_i V_i (x_r = the sum when assign)
template <class T>
void vec_lincomb_dev(long n, const cx<T>* V, long ldv, const GmDev* st, cx<T>* x, hipStream_t s, int nr = 1,
                     long ldr = 0, long ldx = 0, bool assign = false);
// Arnoldi reductions of the device-resident GMRES (RHS with st[r].stop skip)
template <class T>
void vec_multidot_skip(long n, int m, const cx<T>* V, long ldv, const cx<T>* w, void* work, hipStream_t s,
                       RedBatch rb);
// w -= sum_i h_i V_i with h_i = sc_i (stored V_i)^H w summed from the multidot
// partials (written to res + r*ostride), ||w||^2, and then, in the last
// workgroup of each RHS to finish (counter done[r], left at 0), the Givens
// update of column j; w becomes the next basis vector: scaled by the last
// workgroup when `normalize`, else stored as is with sc[j+1] = 1/||w||.
// Stopped RHS are skipped.
template <class T>
void vec_update_norm_givens(long n, int m, const cx<T>* V, long ldv, cx<T>* w, cx<double>* res, void* work,
                            hipStream_t s, RedBatch rb, GmDev* st, int j, int* done, bool normalize);

}  // namespace dd
