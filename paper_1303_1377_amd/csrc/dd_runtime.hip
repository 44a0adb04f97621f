// dd_runtime.hip -- host runtime and C-ABI of the MI355X DD-alpha-AMG solver.
//
//   hierarchy ........ levels, standard aggregation, SAP block colouring (Sec. 2.3, 3.2)
//   outer solver ..... FGMRES(n_kv) in FP64, right-preconditioned by one V-cycle (Sec. 4.2)
//   V-cycle .......... C^(nu): restrict, coarse solve, prolong, nu SAP sweeps (eq. iterationmatrix)
//   coarsest solver .. odd-even preconditioned restarted GMRES (Sec. 5)
//   middle levels .... FGMRES preconditioned by the next V-cycle (recursive two-level method)
//   setup ............ Algorithm 2, DD-alpha-AMG-setup(n_inv, nu), level by level
//
// Krylov vectors live on the device; the small Hessenberg least-squares
// problem (Givens rotations) is solved on the host in FP64 from the inner
// products the reduction kernels return, one transfer per Arnoldi step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ddamg.h"
#include "dd_kernels.h"

using namespace dd;
using zc = std::complex<double>;

namespace {

struct DdError {
    dd_status code;
    std::string msg;
};

#define HIPX(call)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            throw DdError{e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EDEVICE,                          \
                          std::string(#call) + ": " + hipGetErrorString(e_)};                        \
    } while (0)

static void fail(dd_status c, const std::string& m) { throw DdError{c, m}; }

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// device allocation registry of one context
struct Arena {
    std::vector<void*> ptrs;
    long long bytes = 0;
    void* alloc(size_t n) {
        void* p = nullptr;
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(DD_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
        ptrs.push_back(p);
        bytes += (long long)n;
        return p;
    }
    template <class X> X* get(size_t count) { return reinterpret_cast<X*>(alloc(sizeof(X) * count)); }
    void release() {
        for (void* p : ptrs) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
    }
    ~Arena() { release(); }
};

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static Geom make_geom(const int d[4], const int b[4]) {
    Geom g;
    g.lex = 0;
    long vol = 1, bvol = 1;
    for (int mu = 0; mu < 4; mu++) {
        g.d[mu] = d[mu];
        g.b[mu] = b[mu];
        g.lb[mu] = ilog2(b[mu]);
        g.nb[mu] = d[mu] / b[mu];
        vol *= d[mu];
        bvol *= b[mu];
    }
    g.bvh = (int)(bvol / 2);
    g.lbvh = ilog2(g.bvh);
    g.vh = (int)(vol / 2);
    g.nblk = g.nb[0] * g.nb[1] * g.nb[2] * g.nb[3];
    return g;
}

// lexicographic layout of a coarsest lattice with an odd extent (no parity
// structure; the two halves of the canonical order stand in for the parities)
static Geom make_geom_lex(const int d[4]) {
    Geom g;
    g.lex = 1;
    long vol = 1;
    for (int mu = 0; mu < 4; mu++) {
        g.d[mu] = d[mu];
        g.b[mu] = d[mu];
        g.lb[mu] = ilog2(d[mu]);
        g.nb[mu] = 1;
        vol *= d[mu];
    }
    g.vh = (int)(vol / 2);
    g.bvh = g.vh;
    g.lbvh = ilog2(g.vh);
    g.nblk = 1;
    return g;
}

// SAP block validity: extents dividing the lattice with an even block count
// (or one block) per dimension, so that two colours suffice (Sec. 2.3)
static bool valid_sap_blocks(const int d[4], const int b[4]) {
    for (int mu = 0; mu < 4; mu++) {
        if (b[mu] < 1 || d[mu] % b[mu]) return false;
        int n = d[mu] / b[mu];
        if (n != 1 && (n & 1)) return false;
    }
    return true;
}

// layout block validity: powers of two >= 2 dividing the extents; blocks
// that carry SAP must also form a 2-colourable grid (an even count, or one
// block, per dimension).  The coarsest level has no SAP, so any count is fine.
static bool valid_layout(const int d[4], const int b[4], bool need_colouring) {
    for (int mu = 0; mu < 4; mu++) {
        if (!is_pow2(b[mu]) || d[mu] % b[mu]) return false;
        int n = d[mu] / b[mu];
        if (need_colouring && n != 1 && (n & 1)) return false;
        if (b[mu] < 2) return false;
    }
    return true;
}

// Givens-rotation state of one (F)GMRES cycle (host, FP64)
struct Hess {
    int m;
    std::vector<zc> H, cs, sn, g, y;
    explicit Hess(int m_) : m(m_), H((m_ + 1) * m_), cs(m_), sn(m_), g(m_ + 1), y(m_) {}
    void reset(double beta) {
        std::fill(H.begin(), H.end(), zc(0));
        std::fill(g.begin(), g.end(), zc(0));
        g[0] = beta;
    }
    zc& h(int i, int j) { return H[i * m + j]; }
    // column j holds h(0..j, j) and h(j+1, j); returns the new residual estimate
    double rotate(int j) {
        for (int i = 0; i < j; i++) {
            zc a = h(i, j), b = h(i + 1, j);
            h(i, j) = std::conj(cs[i]) * a + std::conj(sn[i]) * b;
            h(i + 1, j) = -sn[i] * a + cs[i] * b;
        }
        zc a = h(j, j), b = h(j + 1, j);
        double den = std::sqrt(std::norm(a) + std::norm(b));
        if (den == 0.0) { cs[j] = 1; sn[j] = 0; }
        else { cs[j] = a / den; sn[j] = b / den; }
        h(j, j) = std::conj(cs[j]) * a + std::conj(sn[j]) * b;
        h(j + 1, j) = 0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = std::conj(cs[j]) * g[j];
        return std::abs(g[j + 1]);
    }
    void solve(int k) {
        for (int i = k - 1; i >= 0; i--) {
            zc s = g[i];
            for (int q = i + 1; q < k; q++) s -= h(i, q) * y[q];
            y[i] = s / h(i, i);
        }
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
template <class T> struct Hier;

// layout of the context's device int words (dflags)
static const int DI_BAD = 0;        // error counter of the last checked step
static const int DI_ONES = 16;      // MAX_RHS words that stay 1: "every RHS active"
static const int DI_GATHER = 32;    // {j, its, stop} of each coarsest-GMRES state
static const int DI_BAR = 120;      // cooperative GMRES: barrier count, generation, abort flag
static const int DI_MASK = 128;     // per level: [cycle mask][current mask], MAX_RHS each
static const int DI_DONE = DI_MASK + 2 * MAX_RHS * DD_MAXLEV;   // coarsest GMRES: finished-workgroup
                                                                 // counts, one per RHS (kept at 0)
static const int DI_WORDS = DI_DONE + MAX_RHS;
// reduction results per right-hand side: pass-1 h (0..32), ||w||^2 (33),
// pass-2 h (34..66), ||w||^2 (67)
static const int RS = 136;
static const int GSTR = 64;   // basis factors per RHS in dd_ctx::dg (a cycle holds at most 33 basis vectors)

struct dd_ctx {
    hipStream_t s = nullptr;
    hipStream_t cap = nullptr;   // private stream the Arnoldi-step graphs are captured on
    int dims[4];
    long vol = 0;
    double m0 = 0, csw = 0;
    std::string err;
    Arena fields;        // gauge/clover (survive reconfiguration)
    Arena levels;        // hierarchy buffers
    double* gauge_canon = nullptr;
    double* clover_canon = nullptr;
    // FP64 fine operator (outer solver) in the current layout
    Geom g0;
    cx<double>* U64 = nullptr;
    double* clov64 = nullptr;
    double* clovinv64 = nullptr;
    // FP32 copies for the preconditioner
    cx<float>* U32 = nullptr;
    float* clov32 = nullptr;
    float* clovinv32 = nullptr;
    // FP16 storage copies (precision 16), in the levels arena
    cx<_Float16>* U16 = nullptr;
    _Float16* clov16 = nullptr;
    _Float16* clovinv16 = nullptr;
    int* dflags = nullptr;          // DI_WORDS device ints
    cx<double>* dred = nullptr;     // MAX_RHS * RS reduction results
    double* dg = nullptr;           // FGMRES basis factors: [nesting level][RHS][GSTR] (squared)
    cx<double>* dy = nullptr;       // MAX_RHS * 32 least-squares solutions
    void* dwork = nullptr;          // reduction partials
    cx<double>* hred = nullptr;     // pinned mirror of dred
    cx<double>* hy = nullptr;       // pinned staging of dy
    int* hint = nullptr;            // pinned mirror of dflags
    dd_params p;
    bool configured = false, have_setup = false;
    std::unique_ptr<Hier<double>> H64;
    std::unique_ptr<Hier<float>> H32;
    double last_setup_s = 0;
    // live kernel timing (dd_profile)
    bool prof_on = false;
    unsigned prof_mask = 0;   // classes timed while prof_on (bit c: class c)
    bool capturing = false;      // a graph capture is in progress (no event records)
    std::vector<hipEvent_t> ev_pool;
    struct Rec { int cls; hipEvent_t a, b; double bytes; };
    std::vector<Rec> pending;
    long prof_n[DD_K_NCLASS] = {0};
    double prof_ms[DD_K_NCLASS] = {0};
    double prof_bytes[DD_K_NCLASS] = {0};
    // FP64 outer workspace for max_rhs right-hand sides
    int R = 1;                 // slots of every batched vector set
    cx<double>* oV = nullptr;  // basis: V_i of RHS r at oV + (i*R + r)*n
    cx<double>* ob = nullptr;  // R right-hand sides
    cx<double>* ox = nullptr;  // R solutions
    cx<double>* ot = nullptr;  // 2R temporaries
    // continuous batching (dd_stream_*): per-slot state of the outer FGMRES
    // between restart cycles; slot r uses the r-th vector of every outer set
    struct StreamSlots {
        int state[MAX_RHS] = {0};   // DD_SLOT_* of include/ddamg.h
        double tol[MAX_RHS] = {0}, beta[MAX_RHS] = {0}, bnorm[MAX_RHS] = {0};
        long its[MAX_RHS] = {0};
        int restarts[MAX_RHS] = {0};
        std::vector<Hess> hs;
        bool any() const {
            for (int r = 0; r < MAX_RHS; r++)
                if (state[r]) return true;
            return false;
        }
    } stream;
    void* bicg_ws = nullptr;     // odd-even BiCGStab vectors (levels arena; cleared with it)
    int bicg_prec = 0;
    void* id_ws = nullptr;       // inexact-deflation vectors (levels arena; cleared with it)
    void* scratch = nullptr;     // device address of this GPU's `scratch` array (dd_apply_D_noalloc)
    std::string scratch_err;     // why it is unavailable, if it is
    int sched = SCHED_LDS | SCHED_XCD | SCHED_GRAPH;   // launch schedule (SCHED_* flags)
    int coop_cap = 32;           // workgroups of the cooperative coarse GMRES (autotuned)
    ~dd_ctx();
};

// The right-hand sides one launch sequence works on: slots 0..nr-1 of every
// vector set, active ones flagged on the device (d[r] = 1) and on the host.
struct Batch {
    int nr;
    int* d;
    unsigned h;
    Mask mask() const { return Mask{d, 1, 0}; }
    int count() const { return __builtin_popcount(h); }
    bool on(int r) const { return (h >> r) & 1u; }
};

static hipEvent_t ev_get(dd_ctx* C) {
    if (C->ev_pool.empty()) {
        hipEvent_t e;
        HIPX(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = C->ev_pool.back();
    C->ev_pool.pop_back();
    return e;
}

// accumulate finished event pairs (the stream has been synchronised)
static void harvest(dd_ctx* C) {
    for (auto& r : C->pending) {
        float ms = 0;
        HIPX(hipEventElapsedTime(&ms, r.a, r.b));
        C->prof_n[r.cls]++;
        C->prof_ms[r.cls] += ms;
        C->prof_bytes[r.cls] += r.bytes;
        C->ev_pool.push_back(r.a);
        C->ev_pool.push_back(r.b);
    }
    C->pending.clear();
}

static void sync(dd_ctx* C) {
    HIPX(hipStreamSynchronize(C->s));
    if (!C->pending.empty()) harvest(C);
}

// brackets the launches issued in its scope with events when profiling is on
// `bytes`: algorithmic device-memory traffic of the bracketed launches
// (every datum the step must read or write, counted once)
struct Prof {
    dd_ctx* C;
    int cls;
    double bytes;
    hipEvent_t a = nullptr;
    Prof(dd_ctx* c, int k, double by = 0) : C(c), cls(k), bytes(by) {
        if (C->prof_on && !C->capturing && ((C->prof_mask >> cls) & 1u)) {
            a = ev_get(C);
            HIPX(hipEventRecord(a, C->s));
        }
    }
    ~Prof() noexcept(false) {
        if (a) {
            hipEvent_t b = ev_get(C);
            HIPX(hipEventRecord(b, C->s));
            C->pending.push_back(dd_ctx::Rec{cls, a, b, bytes});
            if (C->pending.size() > 4096) sync(C);
        }
    }
};

static int read_flag(dd_ctx* C, int idx) {
    HIPX(hipMemcpyAsync(C->hint + idx, C->dflags + idx, sizeof(int), hipMemcpyDeviceToHost, C->s));
    sync(C);
    return C->hint[idx];
}
static void clear_flag(dd_ctx* C, int idx) { HIPX(hipMemsetAsync(C->dflags + idx, 0, sizeof(int), C->s)); }

// copy the reduction results of nr right-hand sides (first `cnt` slots each)
static void read_red(dd_ctx* C, int nr, int cnt) {
    HIPX(hipMemcpyAsync(C->hred, C->dred, sizeof(cx<double>) * ((size_t)(nr - 1) * RS + cnt), hipMemcpyDeviceToHost, C->s));
    sync(C);
}

static Batch single(dd_ctx* C) { return Batch{1, C->dflags + DI_ONES, 1u}; }

// device mask words of `b` at dflags + DI_MASK + word, with host bits h
static Batch with_mask(dd_ctx* C, const Batch& b, int word, unsigned h) {
    Batch o{b.nr, C->dflags + DI_MASK + word, h};
    set_flags(o.d, h, b.nr, C->s);
    return o;
}

// largest cooperative grid of the persistent coarse GMRES for an operator type
template <class Op> struct CoopTypes;
template <class T, class S> struct CoopTypes<CoarseOp<T, S>> {
    static int max_grid() { return coarse_gmres_coop_max_grid<T, S>(); }
};
template <class Op> static int coop_max_grid() {
    static std::once_flag once;
    static int cached = 0;
    std::call_once(once, [] {
        cached = CoopTypes<Op>::max_grid();
        (void)hipGetLastError();
    });
    return cached;
}

// ---------------------------------------------------------------------------
// level hierarchy in preconditioner precision T.  Every level-l vector set has
// R slots (RHS r at base + r*nlv(l)); a Krylov basis stores V_i of RHS r at
// base + (i*R + r)*nlv(l), so basis vector i of a batch is again a vector set.
// ---------------------------------------------------------------------------
template <class T>
struct Hier {
    dd_ctx* C;
    int nlev;
    int R;
    Geom g[DD_MAXLEV];
    int nd[DD_MAXLEV];
    FineOp<T> op0;
    CoarseOp<T> cop[DD_MAXLEV];
    // FP16 storage of the operators the V-cycle applies (precision 16): the
    // fine links and clover blocks, P, D_c and its self-block inverses; the
    // setup builds P and D_c in T and refreshes these copies after each build
    bool half = false;
    FineOp<T, _Float16> op0h;
    CoarseOp<T, _Float16> coph[DD_MAXLEV];
    cx<_Float16>* Ph[DD_MAXLEV];
    cx<_Float16>* Mh[DD_MAXLEV];
    cx<_Float16>* Minvh[DD_MAXLEV];
    cx<_Float16>* Bh[DD_MAXLEV];
    // run f with the fine operator / coarse operator / P of the storage in use
    template <class F> void with_fine(F&& f) {
        if constexpr (std::is_same<T, float>::value)
            if (half) { f(op0h); return; }
        f(op0);
    }
    template <class F> void with_coarse(int l, F&& f) {
        if constexpr (std::is_same<T, float>::value)
            if (half) { f(coph[l]); return; }
        f(cop[l]);
    }
    template <class F> void with_P(int l, F&& f) {
        if constexpr (std::is_same<T, float>::value)
            if (half) { f((const cx<_Float16>*)Ph[l]); return; }
        f((const cx<T>*)P[l]);
    }
    void refresh_half(int l);
    void fold(int l);
    int* blocks[DD_MAXLEV][2];
    int nblocks[DD_MAXLEV][2];
    SapTab stab[DD_MAXLEV];        // SAP blocks that are not layout blocks (bv = 0: they are)
    bool lexl[DD_MAXLEV];          // coarsest level in the lexicographic layout (odd extent):
                                   // plain GMRES on D_c instead of the odd-even form
    AggMap amap[DD_MAXLEV];
    int N[DD_MAXLEV];
    cx<T>* tv[DD_MAXLEV];
    cx<T>* P[DD_MAXLEV];
    cx<T>* M[DD_MAXLEV];
    cx<T>* Minv[DD_MAXLEV];
    cx<T>* B[DD_MAXLEV];    // coarsest level: even-site hop blocks with the self inverse folded in
    cx<T>* rc[DD_MAXLEV];   // restricted residuals on level l (l >= 1)
    cx<T>* ec[DD_MAXLEV];   // coarse corrections on level l (l >= 1)
    cx<T>* wa[DD_MAXLEV];   // scratch sets
    cx<T>* wb[DD_MAXLEV];
    cx<T>* wc[DD_MAXLEV];
    cx<T>* kV[DD_MAXLEV];   // Krylov bases (coarsest GMRES, middle FGMRES)
    cx<T>* kZ[DD_MAXLEV];   // middle FGMRES preconditioned vectors
    int kv_cap[DD_MAXLEV];  // basis vectors kV[l] holds per RHS
    GmDev* gmst[DD_MAXLEV]; // R device GMRES states of the coarsest level
    int last_its[DD_MAXLEV];
    long coarse_count[DD_MAXLEV][MAX_RHS];
    bool coop_off = false;   // the cooperative coarse GMRES failed once on this hierarchy
    // instantiated graphs of one coarsest-level Arnoldi step, by (level, j, nr)
    std::map<long, hipGraphExec_t> graphs;
    ~Hier() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    }

    long nlv(int l) const { return 2L * g[l].vh * nd[l]; }   // complex entries of a level vector

    // algorithmic bytes of one launch for k right-hand sides: operator data
    // once, vector data once per RHS, every datum counted once.  Per fine site:
    // stencil 144 operator reals (links 72, clover 72) + 48 per RHS (in, out);
    // SAP half sweep, per site of the active colour, 144 operator reals + 144
    // per RHS (b, z read and written, the residual, the face values of the
    // neighbouring blocks): 288 reals for one RHS.  Operators stored in FP16
    // (precision 16) count 2 bytes per real, vectors sizeof(T).
    double osz() const { return half ? 2.0 : (double)sizeof(T); }
    double by_dirac(int k) const { return 2.0 * g[0].vh * (144 * osz() + 48.0 * k * sizeof(T)); }
    double by_sap_half(int k) const { return 1.0 * g[0].vh * (144 * osz() + 144.0 * k * sizeof(T)); }
    // FP16 spinor sets: 2 bytes per real and one 4-byte scale per 12 reals
    static constexpr double HSZ = 2.0 + 4.0 / 12.0;
    double by_sap_half_h(int k) const { return 1.0 * g[0].vh * (144 * osz() + 144.0 * k * HSZ); }
    double by_transfer_h(int k) const {
        return (double)nlv(0) * N[0] * 2 * osz() + (double)k * nlv(0) * 2 * HSZ + (double)k * nlv(1) * 2 * sizeof(T);
    }
    double by_coarse(int l, int nblk_per_site, int nvec_per_site, bool all_sites, int k) const {
        double sites = all_sites ? 2.0 * g[l].vh : 1.0 * g[l].vh;
        return sites * ((double)nblk_per_site * nd[l] * nd[l] * 2 * osz() + (double)k * nvec_per_site * nd[l] * 2 * sizeof(T));
    }
    double by_transfer(int l, int k) const {
        // P (N vectors) + fine vector + coarse vector per RHS
        return (double)nlv(l) * N[l] * 2 * osz() + (double)k * nlv(l) * 2 * sizeof(T) +
               (double)k * nlv(l + 1) * 2 * sizeof(T);
    }
    double by_reduce(long n, int m, int k) const { return (double)k * n * (m + 1) * 2 * sizeof(T); }

    Hier(dd_ctx* c) : C(c) {
        memset(blocks, 0, sizeof blocks);
        memset(nblocks, 0, sizeof nblocks);
        memset(tv, 0, sizeof tv);
        memset(P, 0, sizeof P);
        memset(M, 0, sizeof M);
        memset(Minv, 0, sizeof Minv);
        memset(B, 0, sizeof B);
        memset(Bh, 0, sizeof Bh);
        memset(coarse_count, 0, sizeof coarse_count);
        memset(gmst, 0, sizeof gmst);
        memset(kv_cap, 0, sizeof kv_cap);
        memset(Ph, 0, sizeof Ph);
        memset(Mh, 0, sizeof Mh);
        memset(Minvh, 0, sizeof Minvh);
        memset(lexl, 0, sizeof lexl);
        for (int l = 0; l < DD_MAXLEV; l++) {
            last_its[l] = 8;
            stab[l] = SapTab{};
        }
    }

    void build_geometry();
    std::vector<double> norms(long n, const cx<T>* v, long ld, const Batch& b);
    void sap(int l, const cx<T>* b, cx<T>* z, int nsweeps, bool zero_start, const Batch& bt);
    void apply_D(int l, const cx<T>* in, cx<T>* out, const Batch& bt);
    void restrict_(int l, const cx<T>* in, cx<T>* out, const Batch& bt);
    void prolong(int l, const cx<T>* in, cx<T>* out, const Batch& bt);
    void schur(int l, const cx<T>* v, cx<T>* out, Mask mk, int nr, int k);
    void gmres_oe(int l, const cx<T>* r, cx<T>* e, const Batch& bt);
    void fgmres_mid(int l, int bottom, const cx<T>* r, cx<T>* e, const Batch& bt);
    void vcycle(int l, int bottom, const cx<T>* r, cx<T>* z, const Batch& bt);
    // the fine level of the V-cycle on FP16 spinor sets (precision 16)
    void sap(int l, hspin b, hspin z, int nsweeps, bool zero_start, const Batch& bt);
    void restrict_(int l, hspin in, cx<T>* out, const Batch& bt);
    void prolong(int l, const cx<T>* in, hspin out, const Batch& bt);
    void vcycle(int l, int bottom, hspin r, hspin z, const Batch& bt);
    // an FP16 spinor set of R fine vectors in the memory of a level-0 scratch set
    // (R sets of 28 vh four-byte slots: 7/12 of the set's bytes)
    hspin as_h(cx<T>* buf) const { return hspin{reinterpret_cast<hpair*>(buf)}; }
    void build(int l);
    void setup_level(int l, bool given);
    double norm1(long n, const cx<T>* v) { return norms(n, v, 0, single(C))[0]; }
};

dd_ctx::~dd_ctx() {
    H64.reset();
    H32.reset();
    if (cap) (void)hipStreamDestroy(cap);
    for (auto& r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    H64.reset();
    H32.reset();
    levels.release();
    fields.release();
    if (hred) (void)hipHostFree(hred);
    if (hy) (void)hipHostFree(hy);
    if (hint) (void)hipHostFree(hint);
}

// ---------------------------------------------------------------------------
// fine fields: layout import, clover
// ---------------------------------------------------------------------------
static void layout_fields(dd_ctx* C, const int b[4], const double* gauge_src, const double* clover_src) {
    // gauge_src / clover_src are device canonical arrays that stay valid during the call
    Arena fresh;
    double* gcanon = fresh.get<double>((size_t)C->vol * 72);
    HIPX(hipMemcpyAsync(gcanon, gauge_src, sizeof(double) * C->vol * 72, hipMemcpyDeviceToDevice, C->s));
    double* ccanon = nullptr;
    if (clover_src) {
        ccanon = fresh.get<double>((size_t)C->vol * 144);
        HIPX(hipMemcpyAsync(ccanon, clover_src, sizeof(double) * C->vol * 144, hipMemcpyDeviceToDevice, C->s));
    }
    Geom g = make_geom(C->dims, b);
    cx<double>* U64 = fresh.get<cx<double>>((size_t)C->vol * 36);
    double* clov = fresh.get<double>((size_t)C->vol * 72);
    double* clovinv = fresh.get<double>((size_t)C->vol * 72);
    cx<float>* U32 = fresh.get<cx<float>>((size_t)C->vol * 36);
    float* clov32 = fresh.get<float>((size_t)C->vol * 72);
    float* clovinv32 = fresh.get<float>((size_t)C->vol * 72);
    int* flags = fresh.get<int>(DI_WORDS);
    HIPX(hipMemsetAsync(flags, 0, sizeof(int) * DI_WORDS, C->s));
    set_flags(flags + DI_ONES, (1u << MAX_RHS) - 1, MAX_RHS, C->s);
    fine_import_gauge<double>(g, gcanon, U64, C->s);
    fine_import_gauge<float>(g, gcanon, U32, C->s);
    if (ccanon) fine_clover_from_user(g, ccanon, C->m0, clov, clovinv, flags, C->s);
    else fine_clover_from_links(g, U64, C->m0, C->csw, clov, clovinv, flags, C->s);
    vec_convert<float, double>((long)C->vol * 36, reinterpret_cast<const cx<double>*>(clov),
                               reinterpret_cast<cx<float>*>(clov32), C->s);
    vec_convert<float, double>((long)C->vol * 36, reinterpret_cast<const cx<double>*>(clovinv),
                               reinterpret_cast<cx<float>*>(clovinv32), C->s);
    HIPX(hipGetLastError());
    HIPX(hipMemcpyAsync(C->hint, flags, sizeof(int), hipMemcpyDeviceToHost, C->s));
    HIPX(hipStreamSynchronize(C->s));
    const int bad = C->hint[0];
    // swap arenas
    C->fields.release();
    C->fields.ptrs.swap(fresh.ptrs);
    C->fields.bytes = fresh.bytes;
    fresh.bytes = 0;
    C->gauge_canon = gcanon;
    C->clover_canon = ccanon;
    C->g0 = g;
    C->U64 = U64; C->clov64 = clov; C->clovinv64 = clovinv;
    C->U32 = U32; C->clov32 = clov32; C->clovinv32 = clovinv32;
    C->dflags = flags;
    C->dred = C->fields.get<cx<double>>((size_t)MAX_RHS * RS);
    C->dg = C->fields.get<double>((size_t)DD_MAXLEV * MAX_RHS * GSTR);
    C->dy = C->fields.get<cx<double>>((size_t)MAX_RHS * 32);
    C->dwork = C->fields.alloc(reduce_work_size(34, MAX_RHS));
    if (bad) fail(DD_ENUMERIC, "singular clover block on " + std::to_string(bad) + " sites");
}

template <class T> static FineOp<T> fine_op(dd_ctx* C);
template <> FineOp<double> fine_op<double>(dd_ctx* C) {
    return FineOp<double>{C->g0, C->U64, C->clov64, C->clovinv64, C->sched};
}
template <> FineOp<float> fine_op<float>(dd_ctx* C) {
    return FineOp<float>{C->g0, C->U32, C->clov32, C->clovinv32, C->sched};
}

// ---------------------------------------------------------------------------
// hierarchy geometry and buffers
// ---------------------------------------------------------------------------
template <class T>
void Hier<T>::build_geometry() {
    const dd_params& p = C->p;
    nlev = p.levels;
    R = C->R;
    Arena& A = C->levels;
    g[0] = C->g0;
    nd[0] = 12;
    op0 = fine_op<T>(C);
    half = (p.precision == 16);
    if (half) {
        const long vol = 2L * g[0].vh;
        C->U16 = A.get<cx<_Float16>>((size_t)vol * 36);
        C->clov16 = reinterpret_cast<_Float16*>(A.get<cx<_Float16>>((size_t)vol * 36));
        C->clovinv16 = reinterpret_cast<_Float16*>(A.get<cx<_Float16>>((size_t)vol * 36));
        vec_convert<_Float16, float>(vol * 36, C->U32, C->U16, C->s);
        vec_convert<_Float16, float>(vol * 36, reinterpret_cast<const cx<float>*>(C->clov32),
                                     reinterpret_cast<cx<_Float16>*>(C->clov16), C->s);
        vec_convert<_Float16, float>(vol * 36, reinterpret_cast<const cx<float>*>(C->clovinv32),
                                     reinterpret_cast<cx<_Float16>*>(C->clovinv16), C->s);
        op0h = FineOp<T, _Float16>{g[0], C->U16, C->clov16, C->clovinv16, C->sched};
    }
    int d[4];
    memcpy(d, C->dims, sizeof d);
    for (int l = 0; l < nlev; l++) {
        bool sap_tables = false;
        if (l > 0) {
            int b[4];
            bool has_sap = (l < nlev - 1);
            bool all_even = true;
            for (int mu = 0; mu < 4; mu++) all_even = all_even && !(d[mu] & 1);
            if (!has_sap && !all_even) {
                // coarsest lattice with an odd extent: lexicographic layout, plain GMRES
                if (((long)d[0] * d[1] * d[2] * d[3]) & 1)
                    fail(DD_EINVAL, "level " + std::to_string(l) + ": the coarsest lattice needs an even volume");
                g[l] = make_geom_lex(d);
                lexl[l] = true;
            } else {
                for (int mu = 0; mu < 4; mu++) b[mu] = has_sap ? p.sap[l][mu] : 2;
                if (has_sap && !valid_layout(d, b, true) && valid_sap_blocks(d, b) && all_even) {
                    // SAP blocks that are no layout blocks (e.g. 2 x 3^3): layout blocks 2^4, SAP from tables
                    for (int mu = 0; mu < 4; mu++) b[mu] = 2;
                    sap_tables = true;
                }
                if (!valid_layout(d, b, has_sap && !sap_tables))
                    fail(DD_EINVAL, "level " + std::to_string(l) + ": lattice/blocks not supported (SAP blocks must divide "
                                    "the lattice with an even block count per dimension, and a level with SAP needs "
                                    "even extents)");
                g[l] = make_geom(d, b);
            }
            nd[l] = 2 * p.n_tv[l - 1];
            M[l] = A.get<cx<T>>((size_t)2 * g[l].vh * 9 * nd[l] * nd[l]);
            Minv[l] = A.get<cx<T>>((size_t)2 * g[l].vh * nd[l] * nd[l]);
            const bool coarsest = (l == nlev - 1) && nd[l] <= 64 && !lexl[l];
            if (coarsest) B[l] = A.get<cx<T>>((size_t)g[l].vh * 8 * nd[l] * nd[l]);
            cop[l] = CoarseOp<T>{g[l], nd[l], M[l], Minv[l], (C->sched & SCHED_NO_MFMA) ? 0 : 1, B[l]};
            if (half) {
                Mh[l] = A.get<cx<_Float16>>((size_t)2 * g[l].vh * 9 * nd[l] * nd[l]);
                Minvh[l] = A.get<cx<_Float16>>((size_t)2 * g[l].vh * nd[l] * nd[l]);
                if (coarsest) Bh[l] = A.get<cx<_Float16>>((size_t)g[l].vh * 8 * nd[l] * nd[l]);
                coph[l] = CoarseOp<T, _Float16>{g[l], nd[l], Mh[l], Minvh[l], (C->sched & SCHED_NO_MFMA) ? 0 : 1, Bh[l]};
            }
            rc[l] = A.get<cx<T>>((size_t)R * nlv(l));
            ec[l] = A.get<cx<T>>((size_t)R * nlv(l));
        }
        wa[l] = A.get<cx<T>>((size_t)R * nlv(l));
        wb[l] = A.get<cx<T>>((size_t)R * nlv(l));
        wc[l] = A.get<cx<T>>((size_t)R * nlv(l));
        if (l < nlev - 1) {
            // SAP block lists by colour (red = even sum of block coordinates)
            std::vector<int> lists[2];
            const Geom& G = g[l];
            if (sap_tables) {
                // blocks p.sap[l]: per block the layout indices of its even and odd
                // sites (canonical order), per site its block and position
                const int* sb = p.sap[l];
                int nbk[4];
                for (int mu = 0; mu < 4; mu++) nbk[mu] = d[mu] / sb[mu];
                const int nsb = nbk[0] * nbk[1] * nbk[2] * nbk[3];
                std::vector<std::vector<int>> sl(2 * (size_t)nsb);
                const long vol = 2L * G.vh;
                std::vector<int> of(vol), loc(vol);
                for (long c = 0; c < vol; c++) {
                    int x[4];
                    canon_coords(d, c, x);
                    int bc[4];
                    for (int mu = 0; mu < 4; mu++) bc[mu] = x[mu] / sb[mu];
                    const int B = ((bc[0] * nbk[1] + bc[1]) * nbk[2] + bc[2]) * nbk[3] + bc[3];
                    const int par = site_parity(x);
                    const int i = cb_index(G, x);
                    loc[(size_t)par * G.vh + i] = (int)sl[2 * (size_t)B + par].size();
                    of[(size_t)par * G.vh + i] = B;
                    sl[2 * (size_t)B + par].push_back(i);
                }
                const int bv = (int)sl[0].size();
                for (auto& v : sl)
                    if ((int)v.size() != bv)
                        fail(DD_EINVAL, "level " + std::to_string(l) + ": SAP blocks need as many even as odd sites");
                if (bv * nd[l] > 2048) fail(DD_EINVAL, "coarse SAP block too large for one workgroup");
                std::vector<int> sites((size_t)nsb * 2 * bv);
                for (int B = 0; B < nsb; B++)
                    for (int par = 0; par < 2; par++)
                        for (int q = 0; q < bv; q++) sites[((size_t)B * 2 + par) * bv + q] = sl[2 * (size_t)B + par][q];
                int* dsites = A.get<int>(sites.size());
                int* dof = A.get<int>(vol);
                int* dloc = A.get<int>(vol);
                HIPX(hipMemcpyAsync(dsites, sites.data(), sizeof(int) * sites.size(), hipMemcpyHostToDevice, C->s));
                HIPX(hipMemcpyAsync(dof, of.data(), sizeof(int) * vol, hipMemcpyHostToDevice, C->s));
                HIPX(hipMemcpyAsync(dloc, loc.data(), sizeof(int) * vol, hipMemcpyHostToDevice, C->s));
                HIPX(hipStreamSynchronize(C->s));
                stab[l] = SapTab{dsites, dof, dloc, bv};
                for (int B = 0; B < nsb; B++) {
                    int r = B, bc3 = r % nbk[3]; r /= nbk[3];
                    int bc2 = r % nbk[2]; r /= nbk[2];
                    int bc1 = r % nbk[1], bc0 = r / nbk[1];
                    lists[(bc0 + bc1 + bc2 + bc3) & 1].push_back(B);
                }
            } else {
                for (int bi = 0; bi < G.nblk; bi++) {
                    int r = bi, bc3 = r % G.nb[3]; r /= G.nb[3];
                    int bc2 = r % G.nb[2]; r /= G.nb[2];
                    int bc1 = r % G.nb[1], bc0 = r / G.nb[1];
                    lists[(bc0 + bc1 + bc2 + bc3) & 1].push_back(bi);
                }
            }
            for (int c = 0; c < 2; c++) {
                nblocks[l][c] = (int)lists[c].size();
                blocks[l][c] = A.get<int>(lists[c].size() + 1);
                if (!lists[c].empty())
                    HIPX(hipMemcpyAsync(blocks[l][c], lists[c].data(), sizeof(int) * lists[c].size(), hipMemcpyHostToDevice, C->s));
            }
            if (l > 0 && !sap_tables && g[l].bvh * nd[l] > 1024) fail(DD_EINVAL, "coarse SAP block too large for one workgroup");
            // aggregation onto level l+1
            int a[4], dc[4];
            for (int mu = 0; mu < 4; mu++) {
                a[mu] = p.agg[l][mu];
                if (a[mu] <= 0 || d[mu] % a[mu]) fail(DD_EINVAL, "aggregates do not divide level " + std::to_string(l));
                dc[mu] = d[mu] / a[mu];
                // odd extents only on the coarsest level (lexicographic layout, plain GMRES)
                if (dc[mu] < 1 || ((dc[mu] & 1) && l + 1 < nlev - 1))
                    fail(DD_EINVAL, "coarse lattice extents must be even below the coarsest level (level " +
                                        std::to_string(l + 1) + ")");
            }
            N[l] = p.n_tv[l];
            if (N[l] < 1 || N[l] > 32) fail(DD_EINVAL, "n_tv must be in 1..32");
            int asz = a[0] * a[1] * a[2] * a[3];
            if (asz > 1024 || (l > 0 && asz * nd[l] > 1024)) fail(DD_EINVAL, "aggregate too large for one workgroup");
            amap[l].f = g[l];
            amap[l].asz = asz;
            memcpy(amap[l].a, a, sizeof a);
            tv[l] = A.get<cx<T>>((size_t)N[l] * nlv(l));
            P[l] = A.get<cx<T>>((size_t)N[l] * nlv(l));
            if (half) Ph[l] = A.get<cx<_Float16>>((size_t)N[l] * nlv(l));
            memcpy(d, dc, sizeof d);
        }
    }
    for (int l = 0; l + 1 < nlev; l++) amap[l].c = g[l + 1];
    // Krylov workspaces.  A middle level runs FGMRES(mid_restart) in solves,
    // but during the setup of the level above it is the coarsest level of
    // the V-cycle and runs GMRES(coarse_restart): its basis holds the larger.
    for (int l = 1; l < nlev; l++) {
        const int mv = (l == nlev - 1) ? C->p.coarse_restart : std::max(C->p.mid_restart, C->p.coarse_restart);
        kV[l] = A.get<cx<T>>((size_t)(mv + 1) * R * nlv(l));
        kv_cap[l] = mv + 1;
        kZ[l] = (l < nlev - 1) ? A.get<cx<T>>((size_t)C->p.mid_restart * R * nlv(l)) : nullptr;
        gmst[l] = A.get<GmDev>(R);
    }
    HIPX(hipStreamSynchronize(C->s));
}

// ---------------------------------------------------------------------------
// elementary steps (every one over the active right-hand sides of a batch)
// ---------------------------------------------------------------------------
template <class T>
std::vector<double> Hier<T>::norms(long n, const cx<T>* v, long ld, const Batch& b) {
    RedBatch rb{b.nr, ld, ld, RS, b.mask()};
    vec_multidot<T>(n, 1, v, 0, v, C->dred, C->dwork, nullptr, C->s, rb);
    read_red(C, b.nr, 1);
    std::vector<double> out(b.nr, 0.0);
    for (int r = 0; r < b.nr; r++)
        if (b.on(r)) out[r] = std::sqrt(C->hred[(size_t)r * RS].re);
    return out;
}

template <class T>
void Hier<T>::apply_D(int l, const cx<T>* in, cx<T>* out, const Batch& bt) {
    Prof pr(C, l == 0 ? DD_K_DIRAC_PREC : DD_K_COARSE, l == 0 ? by_dirac(bt.count()) : by_coarse(l, 9, 2, true, bt.count()));
    if (l == 0) with_fine([&](auto& op) { fine_dirac(op, in, out, C->s, bt.nr, nlv(0), bt.mask()); });
    else with_coarse(l, [&](auto& op) { coarse_apply(op, -1, CS_SELF, in, 1, in, false, out, C->s, bt.mask(), bt.nr, nlv(l)); });
}

// nsweeps SAP iterations on level l (red blocks, then black blocks)
template <class T>
void Hier<T>::sap(int l, const cx<T>* b, cx<T>* z, int nsweeps, bool zero_start, const Batch& bt) {
    if (zero_start) HIPX(hipMemsetAsync(z, 0, sizeof(cx<T>) * nlv(l) * bt.nr, C->s));
    for (int sw = 0; sw < nsweeps; sw++)
        for (int c = 0; c < 2; c++) {
            Prof pr(C, l == 0 ? DD_K_SAP : DD_K_COARSE_SAP,
                    l == 0 ? by_sap_half(bt.count()) : by_coarse(l, 9, 3, false, bt.count()));
            if (l == 0)
                with_fine([&](auto& op) {
                    fine_sap_half(op, blocks[0][c], nblocks[0][c], b, z, C->p.mr_steps[0], C->s, bt.nr, nlv(0), bt.mask());
                });
            else
                with_coarse(l, [&](auto& op) {
                    coarse_sap_half(op, blocks[l][c], nblocks[l][c], b, z, C->p.mr_steps[l], C->s, bt.nr, nlv(l), bt.mask(),
                                    stab[l]);
                });
        }
}

template <class T>
void Hier<T>::restrict_(int l, const cx<T>* in, cx<T>* out, const Batch& bt) {
    Prof pr(C, DD_K_RESTRICT, by_transfer(l, bt.count()));
    with_P(l, [&](auto* Pl) {
        if (l == 0) fine_restrict(amap[0], N[0], Pl, in, out, C->s, bt.nr, nlv(0), nlv(1), bt.mask());
        else coarse_restrict(amap[l], nd[l], N[l], Pl, in, out, C->s, bt.nr, nlv(l), nlv(l + 1), bt.mask());
    });
}

template <class T>
void Hier<T>::prolong(int l, const cx<T>* in, cx<T>* out, const Batch& bt) {
    Prof pr(C, DD_K_PROLONG, by_transfer(l, bt.count()));
    with_P(l, [&](auto* Pl) {
        if (l == 0) fine_prolong(amap[0], N[0], Pl, in, out, C->s, bt.nr, nlv(1), nlv(0), bt.mask());
        else coarse_prolong(amap[l], nd[l], N[l], Pl, in, out, C->s, bt.nr, nlv(l + 1), nlv(l), bt.mask());
    });
}

// out_o = (A_oo - D_oe A_ee^{-1} D_eo) v_o ; the even part of out is not written
template <class T>
void Hier<T>::schur(int l, const cx<T>* v, cx<T>* out, Mask mk, int nr, int k) {
    // two launches, each over one parity: 8 hop blocks + (Minv | self) per site
    Prof pr(C, DD_K_COARSE, 2 * by_coarse(l, 9, 2, false, k));
    with_coarse(l, [&](auto& op) {
        if (op.B && !coarse_uses_mfma(op, nr)) coarse_apply_folded(op, (const cx<T>*)nullptr, 1, v, wc[l], C->s, mk, nr, nlv(l));
        else coarse_apply(op, 0, CS_NONE, (const cx<T>*)nullptr, 1, v, true, wc[l], C->s, mk, nr, nlv(l));
        coarse_apply(op, 1, CS_SELF, v, -1, wc[l], false, out, C->s, mk, nr, nlv(l));
    });
}

// ---------------------------------------------------------------------------
// coarsest level: odd-even GMRES(m) to relative residual coarse_tol (Sec. 5).
// The Arnoldi bookkeeping lives on the device, one GmDev per right-hand side,
// so the host can enqueue a chunk of Arnoldi steps (sized from the previous
// solve on this level) before it reads back the step counts and stop flags.
// Every kernel of a step skips the right-hand sides whose flag is set, so the
// RHS of a batch advance in lockstep and each one stops on its own residual.
// ---------------------------------------------------------------------------
template <class T>
void Hier<T>::gmres_oe(int l, const cx<T>* r, cx<T>* e, const Batch& bt) {
    const dd_params& p = C->p;
    const int m = p.coarse_restart, nr = bt.nr, k = bt.count();
    if (m + 1 > kv_cap[l] || !gmst[l] || nr > R) fail(DD_EINVAL, "GMRES workspace of level " + std::to_string(l) + " too small");
    const long nfull = nlv(l), nh = (long)g[l].vh * nd[l];
    const long ldv = (long)R * nfull;   // basis stride
    cx<T>* V = kV[l];
    cx<T>* f = wa[l];
    cx<T>* t = wb[l];
    GmDev* st = gmst[l];
    const Mask live{&st->stop, (int)(sizeof(GmDev) / sizeof(int)), 1};
    const Mask in = bt.mask();
    // a coarsest lattice with an odd extent has no odd-even structure: plain
    // GMRES on D_c (Krylov vectors of the full length, no reduction)
    const bool full = lexl[l];
    const long nred = full ? nfull : nh;
    auto odd = [&](cx<T>* v) { return full ? v : v + nh; };
    // A_ee^{-1} D_eo in one pass with the folded blocks (vector-unit forms)
    bool folded = false;
    with_coarse(l, [&](auto& op) { folded = !full && op.B && !coarse_uses_mfma(op, nr); });
    if (full) {
        HIPX(hipMemcpyAsync(f, r, sizeof(cx<T>) * nfull * nr, hipMemcpyDeviceToDevice, C->s));
    } else {
        // t_e = A_ee^{-1} r_e ; f_o = r_o - D_oe t_e
        Prof pr(C, DD_K_COARSE, by_coarse(l, 1, 2, false, k) + by_coarse(l, 8, 3, false, k));
        with_coarse(l, [&](auto& op) {
            coarse_apply(op, 0, CS_SELFINV, r, 0, (const cx<T>*)nullptr, false, t, C->s, in, nr, nfull);
            coarse_apply(op, 1, CS_IDENT, r, -1, t, false, f, C->s, in, nr, nfull);
        });
    }
    // V_0 = f_o / ||f_o||.  The first correction is assigned, so e needs no
    // clearing unless right-hand sides outside the batch's mask keep theirs
    if (k < nr) HIPX(hipMemsetAsync(e, 0, sizeof(cx<T>) * nfull * nr, C->s));
    RedBatch rb0{nr, nfull, nfull, RS, in};
    vec_multidot<T>(nred, 1, odd(f), 0, odd(f), C->dred, C->dwork, nullptr, C->s, rb0);
    gm_start(st, C->dred, RS, p.coarse_tol, 1, m, p.coarse_maxit, p.coarse_fixed, nr, C->s, in);
    vec_scale_dev<T>(nred, st, odd(V), C->s, true, nr, nfull, odd(f));
    bool first_cycle = true;
    int* hs = C->hint + DI_GATHER;
    auto read_state = [&]() {
        gm_gather(st, nr, C->dflags + DI_GATHER, C->s);
        HIPX(hipMemcpyAsync(hs, C->dflags + DI_GATHER, 3 * sizeof(int) * nr, hipMemcpyDeviceToHost, C->s));
        sync(C);
        for (int q = 0; q < nr; q++)
            if (!hs[3 * q + 2]) return false;
        return true;
    };
    const RedBatch rb{nr, nfull, nfull, RS, live};
    // one Arnoldi step of every running RHS, enqueued on stream `sq`
    // (the Prof brackets record nothing while a graph is being captured)
    auto arnoldi_step = [&](int j, hipStream_t sq) {
        cx<T>* vj = V + (size_t)j * ldv;
        cx<T>* w = V + (size_t)(j + 1) * ldv;
        {
            Prof pr(C, DD_K_COARSE, 2 * by_coarse(l, 9, 2, false, k));
            with_coarse(l, [&](auto& op) {
                // vector-unit forms: basis vectors stay unnormalised, their factors
                // scale the stencil's inputs (no pass over w to normalise it)
                if (full) {
                    coarse_apply(op, -1, CS_SELF, vj, 1, vj, false, w, sq, live, nr, nfull);
                } else if (folded) {
                    coarse_apply_folded(op, (const cx<T>*)nullptr, 1, vj, wc[l], sq, live, nr, nfull, InScale{st, j, 2});
                    coarse_apply(op, 1, CS_SELF, vj, -1, wc[l], false, w, sq, live, nr, nfull, InScale{st, j, 1});
                } else {
                    coarse_apply(op, 0, CS_NONE, (const cx<T>*)nullptr, 1, vj, true, wc[l], sq, live, nr, nfull);
                    coarse_apply(op, 1, CS_SELF, vj, -1, wc[l], false, w, sq, live, nr, nfull);
                }
            });
        }
        Prof pr(C, DD_K_REDUCE, 2 * by_reduce(nred, j + 1, k));
        vec_multidot_skip<T>(nred, j + 1, odd(V), ldv, odd(w), C->dwork, sq, rb);
        vec_update_norm_givens<T>(nred, j + 1, odd(V), ldv, odd(w), C->dred, C->dwork, sq, rb, st, j, C->dflags + DI_DONE,
                                  !folded);
    };
    // graphs need a capture stream; live kernel timing brackets single launches
    const bool use_graphs = (C->sched & SCHED_GRAPH) && C->cap;
    // one cooperative launch per restart cycle when the device admits the grid
    int coop_grid = 0;
    if ((C->sched & SCHED_COOP) && !coop_off && !full && nd[l] <= 64 && nr <= 16 && m <= 32) {
        int mx = 0;
        with_coarse(l, [&](auto& op) {
            using OpT = typename std::remove_reference<decltype(op)>::type;
            mx = coop_max_grid<OpT>();
        });
        coop_grid = std::min({mx, std::max(1, g[l].vh), C->coop_cap});
    }
    int chunk = std::min(m, std::max(1, last_its[l] + 2));
    for (;;) {
        int j = 0;
        bool all_stop = false;
        if (coop_grid > 0) {
            unsigned* bar = reinterpret_cast<unsigned*>(C->dflags + DI_BAR);
            HIPX(hipMemsetAsync(C->dflags + DI_BAR, 0, 3 * sizeof(int), C->s));
            // test of the fallback below: with the abort flag already raised the
            // first grid barrier gives up and every workgroup leaves
            if (C->sched & SCHED_COOP_ABORT) HIPX(hipMemsetD32Async((hipDeviceptr_t)(C->dflags + DI_BAR + 2), 1, 1, C->s));
            hipError_t herr = hipSuccess;
            {
                Prof pr(C, DD_K_COARSE_STEP, 0.0);
                with_coarse(l, [&](auto& op) {
                    herr = coarse_gmres_coop(op, V, ldv, nfull, wc[l], st, nr, m, reinterpret_cast<cx<double>*>(C->dwork),
                                             bar, C->dflags + DI_BAR + 2, coop_grid, C->s);
                });
            }
            if (herr == hipSuccess) {
                all_stop = read_state();
                if (read_flag(C, DI_BAR + 2)) {
                    // a barrier wait gave up (workgroups not co-resident): redo this
                    // coarse solve with single launches and keep them from now on
                    coop_off = true;
                    gmres_oe(l, r, e, bt);
                    return;
                }
                j = m;
            } else {
                (void)hipGetLastError();   // not admitted: step-by-step launches from here on
                coop_grid = 0;
            }
        }
        while (j < m) {
            const int jend = std::min(m, j + chunk);
            if (use_graphs) {
                // the chunk of steps as one graph launch (captured once per
                // (level, first step, step count, batch size)); steps past a
                // right-hand side's convergence are no-ops on the device
                const long key = (((long)l * 64 + j) * 64 + (jend - j)) * 64 + nr;
                auto it = graphs.find(key);
                if (it == graphs.end()) {
                    hipGraph_t gr = nullptr;
                    hipGraphExec_t ex = nullptr;
                    HIPX(hipStreamBeginCapture(C->cap, hipStreamCaptureModeThreadLocal));
                    C->capturing = true;
                    for (int q = j; q < jend; q++) arnoldi_step(q, C->cap);
                    C->capturing = false;
                    HIPX(hipStreamEndCapture(C->cap, &gr));
                    hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(gr);
                    HIPX(e);
                    it = graphs.emplace(key, ex).first;
                }
                double by = 0;
                for (int q = j; q < jend; q++) by += 2 * by_coarse(l, 9, 2, false, k) + 2 * by_reduce(nred, q + 1, k);
                Prof pr(C, DD_K_COARSE_STEP, by);
                HIPX(hipGraphLaunch(it->second, C->s));
                j = jend;
            } else {
                for (; j < jend; j++) arnoldi_step(j, C->s);
            }
            if (read_state()) { all_stop = true; break; }
            chunk = 4;
        }
        gm_solve(st, nr, C->s);
        vec_lincomb_dev<T>(nred, odd(V), ldv, st, odd(e), C->s, nr, nfull, nfull, first_cycle);
        first_cycle = false;
        if (all_stop) break;
        // restart the running RHS from their true (Schur) residual
        if (full) {
            Prof pr(C, DD_K_COARSE, by_coarse(l, 9, 2, true, k));
            with_coarse(l, [&](auto& op) { coarse_apply(op, -1, CS_SELF, e, 1, e, false, V, C->s, live, nr, nfull); });
        } else {
            schur(l, e, V, live, nr, k);
        }
        bvec_sub<T>(nred, odd(f), odd(V), odd(V), nfull, nr, live, C->s);
        vec_multidot<T>(nred, 1, odd(V), 0, odd(V), C->dred, C->dwork, nullptr, C->s, rb);
        gm_start(st, C->dred, RS, p.coarse_tol, 0, m, p.coarse_maxit, p.coarse_fixed, nr, C->s);
        vec_scale_dev<T>(nred, st, odd(V), C->s, false, nr, nfull);
        if (read_state()) break;
        chunk = 4;
    }
    // e_e = A_ee^{-1} (r_e - D_eo e_o)  (= t_e - B e_o with the folded blocks)
    if (!full) {
        Prof pr(C, DD_K_COARSE, by_coarse(l, 9, 2, false, k));
        with_coarse(l, [&](auto& op) {
            if (folded) coarse_apply_folded(op, (const cx<T>*)t, -1, e, e, C->s, in, nr, nfull);
            else coarse_apply(op, 0, CS_IDENT, r, -1, e, true, e, C->s, in, nr, nfull);
        });
    }
    int mx = 0;
    for (int q = 0; q < nr; q++) {
        coarse_count[l][q] += hs[3 * q + 1];
        mx = std::max(mx, hs[3 * q + 1]);
    }
    last_its[l] = mx;
}

// ---------------------------------------------------------------------------
// FGMRES(m) shared by the outer solver (FP64, level 0) and the middle levels
// (precision T): k independent right-preconditioned Krylov processes in
// lockstep with host-side Givens rotations, classical Gram-Schmidt with one
// reorthogonalisation pass, and a true-residual restart.
// ---------------------------------------------------------------------------
struct KrylovResult {
    long its[MAX_RHS];
    int restarts[MAX_RHS];
    double relres[MAX_RHS];
    bool conv[MAX_RHS];
};

// Ops with prec_copy(w) take the next preconditioner input as an FP32 copy
// that the last Gram-Schmidt pass writes while it leaves w final
template <class Ops, class = void>
struct HasPrecCopy : std::false_type {};
template <class Ops>
struct HasPrecCopy<Ops, std::void_t<decltype(std::declval<Ops&>().prec_copy((const void*)nullptr))>> : std::true_type {};

// Ops supplies, for a batch: precond(j, V_j, Z_j, batch), matvec(Z_j -> w),
// residual(x -> V_0 := r - A x over the batch) and the vector sets.
//
// One restart cycle of the right-hand sides in `cyc`: V_0 of each holds its
// current residual, of norm beta[r] > 0.  Up to m Arnoldi steps (a RHS leaves
// when its estimate reaches tol[r] * bnorm[r], at maxit or at `fixed`
// iterations), x += Z y, then the true residual replaces V_0 and beta[r].
// its[r] counts the iterations of RHS r over all cycles.
template <class VS, class ZS, class Ops>
static void fgmres_cycle(dd_ctx* C, Ops& ops, long n, long ldv, int m, const double* tol, int maxit, long fixed,
                         const Batch& in, int word, unsigned cyc, std::vector<Hess>& hs, double* beta,
                         const double* bnorm, long* its) {
    const int nr = in.nr;
    cx<VS>* V = ops.V();
    cx<ZS>* Z = ops.Z();
    Batch bc = with_mask(C, in, word, cyc);
    // The basis is stored unnormalised: V_i = f_i * stored_i, f_i = 1 / |stored_i|
    // (the Arnoldi vector as the Gram-Schmidt passes leave it), which saves a
    // pass over every new vector.  The preconditioners are scale invariant, so
    // the stored Z holds Z_i / f_i, and every coefficient is rescaled: the
    // Hessenberg entries (host), the Gram-Schmidt updates (device factors
    // g_i = f_i^2 in dg, one block per nesting level) and the solution update.
    double* g = C->dg + (size_t)(word / (2 * MAX_RHS)) * MAX_RHS * GSTR;
    std::vector<std::vector<double>> f(nr, std::vector<double>(m + 1, 0.0));
    Coefs g0{};
    for (int r = 0; r < nr; r++)
        if ((cyc >> r) & 1u) {
            hs[r].reset(beta[r]);
            f[r][0] = 1.0 / beta[r];
            g0.v[r] = f[r][0] * f[r][0];
        }
    set_factor(g, GSTR, 0, g0, nr, bc.mask(), C->s);
    Batch cur = with_mask(C, in, word + MAX_RHS, cyc);
    int jend[MAX_RHS] = {0};
    int jmax = 0;
    for (int j = 0; j < m && cur.h; j++) {
        cx<VS>* vj = V + (size_t)j * ldv;
        cx<VS>* w = V + (size_t)(j + 1) * ldv;
        cx<ZS>* zj = Z + (size_t)j * ldv;
        ops.precond(vj, zj, cur);
        ops.matvec(zj, w, cur);
        {
            RedBatch rb{nr, n, n, RS, cur.mask()};
            Prof pr(C, DD_K_REDUCE, (j + 1 <= 16 ? 3.0 : 4.0) * cur.count() * n * (j + 2) * sizeof(cx<VS>));
            // CGS with one reorthogonalisation; the first update and the second
            // pass's inner products share one sweep over the basis where it fits
            vec_multidot<VS>(n, j + 1, V, ldv, w, C->dred, C->dwork, nullptr, C->s, rb);
            if (!vec_update_dot<VS>(n, j + 1, V, ldv, C->dred, w, C->dred + 34, C->dwork, C->s, rb, g, GSTR)) {
                vec_update_norm<VS>(n, j + 1, V, ldv, C->dred, w, C->dred + 33, C->dwork, nullptr, C->s, rb, g, GSTR);
                vec_multidot<VS>(n, j + 1, V, ldv, w, C->dred + 34, C->dwork, nullptr, C->s, rb);
            }
            cx<float>* wc = nullptr;
            if constexpr (HasPrecCopy<Ops>::value) wc = ops.prec_copy(w);
            vec_update_norm<VS>(n, j + 1, V, ldv, C->dred + 34, w, C->dred + 67, C->dwork, nullptr, C->s, rb, g, GSTR,
                                wc, n);
        }
        read_red(C, nr, 68);
        unsigned next = cur.h;
        Coefs gn{};
        for (int r = 0; r < nr; r++) {
            if (!cur.on(r)) continue;
            const cx<double>* h = C->hred + (size_t)r * RS;
            Hess& H = hs[r];
            const double fj = f[r][j];
            for (int i = 0; i <= j; i++)
                H.h(i, j) = (f[r][i] * fj) * zc(h[i].re + h[34 + i].re, h[i].im + h[34 + i].im);
            double hn = std::sqrt(h[67].re);
            if (!std::isfinite(hn)) fail(DD_ENUMERIC, "non-finite Arnoldi coefficient");
            H.h(j + 1, j) = fj * hn;
            double res = H.rotate(j);
            its[r]++;
            jend[r] = j + 1;
            jmax = std::max(jmax, j + 1);
            bool stop;
            if (fixed > 0) stop = its[r] >= fixed;
            else stop = res <= tol[r] * bnorm[r] || its[r] >= maxit;
            if (hn == 0) stop = true;
            if (stop) {
                next &= ~(1u << r);
            } else {
                f[r][j + 1] = 1.0 / hn;
                gn.v[r] = f[r][j + 1] * f[r][j + 1];
            }
        }
        if (next != cur.h) cur = with_mask(C, in, word + MAX_RHS, next);
        if (next) set_factor(g, GSTR, j + 1, gn, nr, cur.mask(), C->s);
    }
    // x += Z y per RHS over the columns of its own cycle (Z_i = f_i * stored Z_i)
    for (int r = 0; r < nr; r++) {
        cx<double>* y = C->hy + (size_t)r * 32;
        if (!bc.on(r)) continue;
        hs[r].solve(jend[r]);
        for (int i = 0; i < jend[r]; i++) y[i] = cx<double>{f[r][i] * hs[r].y[i].real(), f[r][i] * hs[r].y[i].imag()};
    }
    HIPX(hipMemcpyAsync(C->dy, C->hy, sizeof(cx<double>) * 32 * nr, hipMemcpyHostToDevice, C->s));
    Counts jc{};
    for (int r = 0; r < nr; r++) jc.v[r] = jend[r];
    ops.update(jmax, Z, ldv, C->dy, bc, jc);
    // true residual of the cycle's RHS: restart vector and convergence test
    ops.residual(bc);
    std::vector<double> nb = ops.norms(V, bc);
    for (int r = 0; r < nr; r++) {
        if (!bc.on(r)) continue;
        beta[r] = nb[r];
        if (!std::isfinite(beta[r])) fail(DD_ENUMERIC, "non-finite residual");
    }
}

// Restart cycles until every RHS of the batch converged or reached its limit.
template <class VS, class ZS, class Ops>
static void fgmres_batch(dd_ctx* C, Ops& ops, long n, long ldv, int m, double tol, int maxit, long fixed,
                         const Batch& in, int word, const std::vector<double>& bnorm, KrylovResult& out) {
    const int nr = in.nr;
    std::vector<Hess> hs(nr, Hess(m));
    std::vector<double> beta(bnorm);
    std::vector<double> tols(nr, tol);
    unsigned alive = 0;
    for (int r = 0; r < nr; r++) {
        out.its[r] = 0;
        out.restarts[r] = 0;
        out.relres[r] = (in.on(r) && bnorm[r] > 0) ? 1.0 : 0.0;
        out.conv[r] = !in.on(r) || bnorm[r] == 0;
        if (in.on(r) && bnorm[r] > 0) alive |= 1u << r;
    }
    for (;;) {
        // which RHS run another cycle
        unsigned cyc = 0;
        for (int r = 0; r < nr; r++) {
            if (!((alive >> r) & 1u)) continue;
            out.relres[r] = beta[r] / bnorm[r];
            if (beta[r] <= tol * bnorm[r]) { out.conv[r] = true; continue; }
            if (fixed > 0 ? out.its[r] >= fixed : out.its[r] >= maxit) continue;
            cyc |= 1u << r;
        }
        alive = cyc;
        if (!cyc) break;
        fgmres_cycle<VS, ZS>(C, ops, n, ldv, m, tols.data(), maxit, fixed, in, word, cyc, hs, beta.data(),
                             bnorm.data(), out.its);
        for (int r = 0; r < nr; r++) {
            if (!((cyc >> r) & 1u)) continue;
            out.relres[r] = beta[r] / bnorm[r];
            if (fixed > 0 && out.its[r] >= fixed) {
                out.conv[r] = beta[r] <= tol * bnorm[r];
                alive &= ~(1u << r);
            } else if (beta[r] > tol * bnorm[r]) {
                out.restarts[r]++;
            }
        }
    }
}

// middle levels: FGMRES(m) on D_c preconditioned by the V-cycle of level l
template <class T>
struct MidOps {
    Hier<T>* H;
    int l, bottom;
    const cx<T>* r;
    cx<T>* e;
    cx<T>* V() { return H->kV[l]; }
    cx<T>* Z() { return H->kZ[l]; }
    void precond(const cx<T>* v, cx<T>* z, const Batch& b) { H->vcycle(l, bottom, v, z, b); }
    void matvec(const cx<T>* z, cx<T>* w, const Batch& b) { H->apply_D(l, z, w, b); }
    void update(int m, const cx<T>* Z, long ldz, const cx<double>* y, const Batch& b, const Counts& jc) {
        const long n = H->nlv(l);
        vec_lincomb<T, T>(n, m, Z, ldz, y, e, H->C->s, b.nr, n, 32, n, b.mask(), &jc);
    }
    void residual(const Batch& b) {
        const long n = H->nlv(l);
        H->apply_D(l, e, H->kV[l], b);
        bvec_sub<T>(n, r, H->kV[l], H->kV[l], n, b.nr, b.mask(), H->C->s);
    }
    std::vector<double> norms(const cx<T>* v, const Batch& b) { return H->norms(H->nlv(l), v, H->nlv(l), b); }
};

template <class T>
void Hier<T>::fgmres_mid(int l, int bottom, const cx<T>* r, cx<T>* e, const Batch& bt) {
    const dd_params& p = C->p;
    const long n = nlv(l);
    if (p.mid_restart + 1 > kv_cap[l] || !kZ[l] || bt.nr > R)
        fail(DD_EINVAL, "FGMRES workspace of level " + std::to_string(l) + " too small");
    HIPX(hipMemsetAsync(e, 0, sizeof(cx<T>) * n * bt.nr, C->s));
    std::vector<double> bn = norms(n, r, n, bt);
    HIPX(hipMemcpyAsync(kV[l], r, sizeof(cx<T>) * n * bt.nr, hipMemcpyDeviceToDevice, C->s));
    MidOps<T> ops{this, l, bottom, r, e};
    KrylovResult res;
    fgmres_batch<T, T>(C, ops, n, (long)R * n, p.mid_restart, p.mid_tol, p.mid_maxit, p.mid_fixed, bt,
                               2 * MAX_RHS * l, bn, res);
    for (int q = 0; q < bt.nr; q++) coarse_count[l][q] += res.its[q];
}

// ---------------------------------------------------------------------------
// V-cycle: z = P e_c with e_c ~ D_c^{-1} P^H r, then nu SAP iterations
// ---------------------------------------------------------------------------
template <class T>
void Hier<T>::vcycle(int l, int bottom, const cx<T>* r, cx<T>* z, const Batch& bt) {
    restrict_(l, r, rc[l + 1], bt);
    if (l + 1 == bottom) gmres_oe(l + 1, rc[l + 1], ec[l + 1], bt);
    else fgmres_mid(l + 1, bottom, rc[l + 1], ec[l + 1], bt);
    prolong(l, ec[l + 1], z, bt);
    sap(l, r, z, C->p.nu, false, bt);
}

// ---------------------------------------------------------------------------
// the fine level on FP16 spinor sets (precision 16): the vectors the V-cycle
// reads and writes there (its input r, the interpolated and smoothed z) are
// stored in FP16 with a scale per site and chirality half; arithmetic stays
// FP32 and the coarse levels keep FP32 vectors
// ---------------------------------------------------------------------------
template <class T>
void Hier<T>::sap(int l, hspin b, hspin z, int nsweeps, bool zero_start, const Batch& bt) {
    if constexpr (std::is_same<T, float>::value) {
        if (l != 0 || !half) fail(DD_EINVAL, "FP16 spinor sets on the fine level of precision 16 only");
        if (zero_start) HIPX(hipMemsetAsync(z.d, 0, sizeof(hpair) * (nlv(0) / 6 * 7) * bt.nr, C->s));
        for (int sw = 0; sw < nsweeps; sw++)
            for (int c = 0; c < 2; c++) {
                Prof pr(C, DD_K_SAP, by_sap_half_h(bt.count()));
                with_fine([&](auto& op) {
                    fine_sap_half_h(op, blocks[0][c], nblocks[0][c], b, z, C->p.mr_steps[0], C->s, bt.nr, nlv(0),
                                    bt.mask());
                });
            }
    } else {
        fail(DD_EINVAL, "FP16 spinor sets on the fine level of precision 16 only");
    }
}

template <class T>
void Hier<T>::restrict_(int l, hspin in, cx<T>* out, const Batch& bt) {
    if constexpr (std::is_same<T, float>::value) {
        if (l != 0 || !half) fail(DD_EINVAL, "FP16 spinor sets on the fine level of precision 16 only");
        Prof pr(C, DD_K_RESTRICT, by_transfer_h(bt.count()));
        with_P(0, [&](auto* Pl) { fine_restrict_h(amap[0], N[0], Pl, in, out, C->s, bt.nr, nlv(0), nlv(1), bt.mask()); });
    } else {
        fail(DD_EINVAL, "FP16 spinor sets on the fine level of precision 16 only");
    }
}

template <class T>
void Hier<T>::prolong(int l, const cx<T>* in, hspin out, const Batch& bt) {
    if constexpr (std::is_same<T, float>::value) {
        if (l != 0 || !half) fail(DD_EINVAL, "FP16 spinor sets on the fine level of precision 16 only");
        Prof pr(C, DD_K_PROLONG, by_transfer_h(bt.count()));
        with_P(0, [&](auto* Pl) { fine_prolong_h(amap[0], N[0], Pl, in, out, C->s, bt.nr, nlv(1), nlv(0), bt.mask()); });
    } else {
        fail(DD_EINVAL, "FP16 spinor sets on the fine level of precision 16 only");
    }
}

template <class T>
void Hier<T>::vcycle(int l, int bottom, hspin r, hspin z, const Batch& bt) {
    restrict_(l, r, rc[l + 1], bt);
    if (l + 1 == bottom) gmres_oe(l + 1, rc[l + 1], ec[l + 1], bt);
    else fgmres_mid(l + 1, bottom, rc[l + 1], ec[l + 1], bt);
    prolong(l, ec[l + 1], z, bt);
    sap(l, r, z, C->p.nu, false, bt);
}

// ---------------------------------------------------------------------------
// P, D_c and self-block inverses from the current test vectors of level l
// ---------------------------------------------------------------------------
template <class T>
void Hier<T>::build(int l) {
    clear_flag(C, DI_BAD);
    if (l == 0) fine_gram_schmidt<T>(amap[0], N[0], tv[0], P[0], C->dflags + DI_BAD, C->s);
    else coarse_gram_schmidt<T>(amap[l], nd[l], N[l], tv[l], P[l], C->dflags + DI_BAD, C->s);
    HIPX(hipGetLastError());
    if (read_flag(C, DI_BAD)) fail(DD_ENUMERIC, "rank-deficient aggregate on level " + std::to_string(l));
    if (l == 0) fine_assemble<T>(op0, amap[0], N[0], P[0], M[1], C->s);
    else coarse_assemble<T>(cop[l], amap[l], N[l], P[l], M[l + 1], C->s);
    HIPX(hipGetLastError());
    coarse_self_inverse<T>(g[l + 1], nd[l + 1], M[l + 1], Minv[l + 1], C->dflags + DI_BAD, C->s);
    HIPX(hipGetLastError());
    if (read_flag(C, DI_BAD)) fail(DD_ENUMERIC, "singular coarse self block on level " + std::to_string(l + 1));
    fold(l + 1);
    refresh_half(l);
}

// the folded even-site blocks B_k = Minv M_{1+k} of level l (if it keeps them)
template <class T>
void Hier<T>::fold(int l) {
    if (!B[l]) return;
    coarse_fold_inverse<T>(g[l], nd[l], M[l], Minv[l], B[l], C->s);
    HIPX(hipGetLastError());
}

// FP16 copies of P of level l and of the operator of level l+1
template <class T>
void Hier<T>::refresh_half(int l) {
    if constexpr (std::is_same<T, float>::value) {
        if (!half) return;
        const size_t nn = (size_t)nd[l + 1] * nd[l + 1], vc = 2L * g[l + 1].vh;
        if (Ph[l]) vec_convert<_Float16, float>((long)N[l] * nlv(l), P[l], Ph[l], C->s);
        vec_convert<_Float16, float>((long)(vc * 9 * nn), M[l + 1], Mh[l + 1], C->s);
        vec_convert<_Float16, float>((long)(vc * nn), Minv[l + 1], Minvh[l + 1], C->s);
        if (Bh[l + 1]) vec_convert<_Float16, float>((long)(g[l + 1].vh * 8 * nn), B[l + 1], Bh[l + 1], C->s);
    }
    (void)l;
}

// Algorithm 2 on level l with level l+1 as the coarsest level of its V-cycles
// (with id_setup, the inexact-deflation setup of Sec. 4.3, which replaces the
// update of the second half).  Readings: vectors normalised after each of the
// three initial SAP passes; P and D_c rebuilt from the final vectors.
template <class T>
void Hier<T>::setup_level(int l, bool given) {
    const long n = nlv(l);
    const Batch one = single(C);
    if (!given) {
        if (l == 0) fine_random<T>(g[0], N[0], C->p.seed, l, tv[0], C->s);
        else coarse_random<T>(g[l], nd[l], N[l], C->p.seed, l, tv[l], C->s);
    }
    for (int eta = 1; eta <= 3; eta++)
        for (int j = 0; j < N[l]; j++) {
            cx<T>* v = tv[l] + (size_t)j * n;
            sap(l, v, wa[l], eta, true, one);
            double nv = norm1(n, wa[l]);
            if (!(nv > 0) || !std::isfinite(nv)) fail(DD_ENUMERIC, "setup: vanishing or non-finite test vector");
            HIPX(hipMemcpyAsync(v, wa[l], sizeof(cx<T>) * n, hipMemcpyDeviceToDevice, C->s));
            vec_scale<T>(n, cx<double>{1.0 / nv, 0.0}, v, C->s);
        }
    for (int it = 0; it < C->p.n_inv; it++) {
        build(l);
        for (int j = 0; j < N[l]; j++) {
            cx<T>* v = tv[l] + (size_t)j * n;
            if (C->p.id_setup) {
                // inexact-deflation setup (Sec. 4.3): v_j <- C^(nu) v_j from a zero start
                vcycle(l, l + 1, v, wb[l], one);
                HIPX(hipMemcpyAsync(v, wb[l], sizeof(cx<T>) * n, hipMemcpyDeviceToDevice, C->s));
            } else {
                apply_D(l, v, wa[l], one);
                vec_sub<T>(n, v, wa[l], wa[l], C->s);
                vcycle(l, l + 1, wa[l], wb[l], one);
                vec_axpy<T>(n, cx<double>{1.0, 0.0}, wb[l], v, C->s);
            }
            double nv = norm1(n, v);
            if (!(nv > 0) || !std::isfinite(nv)) fail(DD_ENUMERIC, "setup: vanishing or non-finite test vector");
            vec_scale<T>(n, cx<double>{1.0 / nv, 0.0}, v, C->s);
        }
    }
    build(l);
}

// ---------------------------------------------------------------------------
// outer FGMRES in FP64 with the T-precision V-cycle as right preconditioner
// ---------------------------------------------------------------------------
template <class T>
struct OuterOps {
    dd_ctx* C;
    Hier<T>* H;
    const cx<double>* b;
    cx<double>* x;
    long n;
    cx<T>* Zb;
    cx<double>* V() { return C->oV; }
    cx<T>* Z() { return Zb; }
    cx<T>* vT() { return reinterpret_cast<cx<T>*>(C->ot); }    // preconditioner-precision copies of v_j
    cx<double>* t64() { return C->ot + (size_t)C->R * n; }
    // the FP32 preconditioner takes its input from the Gram-Schmidt pass that
    // finished the vector (fgmres_cycle passes vT() to it): no conversion pass
    const void* copied = nullptr;
    cx<float>* prec_copy(const void* w) {
        if constexpr (std::is_same<T, float>::value) {
            copied = w;
            return vT();
        }
        return nullptr;
    }
    void precond(const cx<double>* v, cx<T>* z, const Batch& bt) {
        if (v != copied) {
            Prof pr(C, DD_K_BLAS, (double)bt.count() * n * (16 + 2 * sizeof(T)));
            bvec_convert<T, double>(n, v, vT(), n, bt.nr, bt.mask(), C->s);
        }
        copied = nullptr;
        H->vcycle(0, H->nlev - 1, vT(), z, bt);
    }
    void matvec(const cx<T>* z, cx<double>* w, const Batch& bt) {
        if constexpr (std::is_same<T, float>::value) {
            // the FP64 stencil reads the FP32 vectors directly
            Prof pr(C, DD_K_DIRAC64, 2.0 * C->g0.vh * (144 * 8 + (24.0 * 4 + 24.0 * 8) * bt.count()));
            fine_dirac_from32(fine_op<double>(C), z, w, C->s, bt.nr, n, bt.mask());
        } else {
            Prof pr(C, DD_K_DIRAC64, 2.0 * C->g0.vh * (144 + 48.0 * bt.count()) * 8);
            fine_dirac<double>(fine_op<double>(C), z, w, C->s, bt.nr, n, bt.mask());
        }
    }
    void update(int m, const cx<T>* Z, long ldz, const cx<double>* y, const Batch& bt, const Counts& jc) {
        vec_lincomb<T, double>(n, m, Z, ldz, y, x, C->s, bt.nr, n, 32, n, bt.mask(), &jc);
    }
    void residual(const Batch& bt) {
        fine_dirac<double>(fine_op<double>(C), x, t64(), C->s, bt.nr, n, bt.mask());
        bvec_sub<double>(n, b, t64(), C->oV, n, bt.nr, bt.mask(), C->s);
    }
    std::vector<double> norms(const cx<double>* v, const Batch& bt) { return norms64(C, n, v, bt); }
    static std::vector<double> norms64(dd_ctx* C, long n, const cx<double>* v, const Batch& bt) {
        RedBatch rb{bt.nr, n, n, RS, bt.mask()};
        vec_multidot<double>(n, 1, v, 0, v, C->dred, C->dwork, nullptr, C->s, rb);
        read_red(C, bt.nr, 1);
        std::vector<double> out(bt.nr, 0.0);
        for (int r = 0; r < bt.nr; r++)
            if (bt.on(r)) out[r] = std::sqrt(C->hred[(size_t)r * RS].re);
        return out;
    }
};

// The outer FGMRES of precision 16: its preconditioned vectors Z and the
// V-cycle's input are FP16 spinor sets.  The Krylov loop addresses Z_j as
// Zb + j ldv in units of cx<_Float16>; zh() turns such an address into the
// FP16 set at the same logical offset (7/12 of the Z area's bytes are used).
// The input lives at the start of C->ot.
struct OuterOpsH {
    dd_ctx* C;
    Hier<float>* H;
    const cx<double>* b;
    cx<double>* x;
    long n;
    int m;
    cx<_Float16>* Zb;
    cx<double>* V() { return C->oV; }
    cx<_Float16>* Z() { return Zb; }
    hspin zh(const cx<_Float16>* z) const { return hspin{reinterpret_cast<hpair*>(Zb)} + (long)(z - Zb); }
    hspin vT() { return hspin{reinterpret_cast<hpair*>(C->ot)}; }
    cx<double>* t64() { return C->ot + (size_t)C->R * n; }
    int vh() const { return (int)(n / 24); }
    void precond(const cx<double>* v, cx<_Float16>* z, const Batch& bt) {
        {
            Prof pr(C, DD_K_BLAS, (double)bt.count() * n * (16 + 2 * Hier<float>::HSZ));
            fine_hpack<double>(vh(), v, vT(), n, bt.nr, bt.mask(), C->s);
        }
        H->vcycle(0, H->nlev - 1, vT(), zh(z), bt);
    }
    void matvec(const cx<_Float16>* z, cx<double>* w, const Batch& bt) {
        {
            Prof pr(C, DD_K_BLAS, (double)bt.count() * n * (16 + 2 * Hier<float>::HSZ));
            fine_hunpack<double>(vh(), zh(z), t64(), n, bt.nr, bt.mask(), C->s);
        }
        Prof pr(C, DD_K_DIRAC64, 2.0 * C->g0.vh * (144 + 48.0 * bt.count()) * 8);
        fine_dirac<double>(fine_op<double>(C), t64(), w, C->s, bt.nr, n, bt.mask());
    }
    void update(int mm, const cx<_Float16>* Z, long ldz, const cx<double>* y, const Batch& bt, const Counts& jc) {
        fine_hlincomb(vh(), mm, zh(Z), ldz, y, x, C->s, bt.nr, n, 32, n, bt.mask(), &jc);
    }
    void residual(const Batch& bt) {
        fine_dirac<double>(fine_op<double>(C), x, t64(), C->s, bt.nr, n, bt.mask());
        bvec_sub<double>(n, b, t64(), C->oV, n, bt.nr, bt.mask(), C->s);
    }
    std::vector<double> norms(const cx<double>* v, const Batch& bt) { return OuterOps<float>::norms64(C, n, v, bt); }
};

// run f(ops, ZS*) with the outer FGMRES operations of the hierarchy (ZS: the
// element type of the preconditioned vectors)
template <class T, class F>
static void with_outer_ops(dd_ctx* C, Hier<T>& H, F&& f) {
    const int m = C->p.outer_restart;
    const long n = 24L * C->g0.vh, ldv = (long)C->R * n;
    if constexpr (std::is_same<T, float>::value) {
        if (H.half) {
            cx<_Float16>* Zb = reinterpret_cast<cx<_Float16>*>(C->oV + (size_t)(m + 1) * ldv);
            OuterOpsH ops{C, &H, C->ob, C->ox, n, m, Zb};
            f(ops, (_Float16*)nullptr);
            return;
        }
    }
    OuterOps<T> ops{C, &H, C->ob, C->ox, n, reinterpret_cast<cx<T>*>(C->oV + (size_t)(m + 1) * ldv)};
    f(ops, (T*)nullptr);
}

// Solve the nr right-hand sides at C->ob into C->ox.
template <class T>
static void outer_fgmres(dd_ctx* C, Hier<T>& H, int nr, double tol, long fixed, dd_stats* st, dd_status* rc) {
    const dd_params& p = C->p;
    const int m = p.outer_restart;
    const long n = 24L * C->g0.vh;
    const long ldv = (long)C->R * n;
    memset(H.coarse_count, 0, sizeof H.coarse_count);
    HIPX(hipMemsetAsync(C->ox, 0, sizeof(cx<double>) * n * nr, C->s));
    clear_flag(C, DI_BAD);
    vec_finite_check<double>(n * nr, C->ob, C->dflags + DI_BAD, C->s);
    if (read_flag(C, DI_BAD)) fail(DD_ENUMERIC, "NaN/Inf in a right-hand side");
    Batch all{nr, C->dflags + DI_ONES, (nr >= 32) ? ~0u : ((1u << nr) - 1)};
    std::vector<double> bn = OuterOps<T>::norms64(C, n, C->ob, all);
    HIPX(hipMemcpyAsync(C->oV, C->ob, sizeof(cx<double>) * n * nr, hipMemcpyDeviceToDevice, C->s));
    KrylovResult res;
    with_outer_ops(C, H, [&](auto& ops, auto* zs) {
        using ZS = std::remove_pointer_t<decltype(zs)>;
        fgmres_batch<double, ZS>(C, ops, n, ldv, m, tol, p.outer_maxit, fixed, all, 0, bn, res);
    });
    for (int r = 0; r < nr; r++) {
        rc[r] = res.conv[r] ? DD_OK : DD_ENOCONV;
        if (!st) continue;
        st[r].outer_iters = (int)res.its[r];
        st[r].restarts = res.restarts[r];
        for (int l = 0; l < DD_MAXLEV; l++) st[r].coarse_iters[l] = H.coarse_count[l][r];
        st[r].true_relres = res.relres[r];
        st[r].converged = res.conv[r] ? 1 : 0;
    }
}


// ---------------------------------------------------------------------------
// Comparison solver of Sec. 6 (Table 3): FGMRES(n_kv) in FP64 right-
// preconditioned by a fixed number of BiCGStab steps (van der Vorst's
// recurrence, zero start) on the odd-even reduced system
//   S x_o = f_o,  S = A_oo - D_oe A_ee^{-1} D_eo,  f_o = b_o - D_oe A_ee^{-1} b_e,
// followed by x_e = A_ee^{-1} (b_e - D_eo x_o), in precision T (FP32 in the
// paper's mixed-precision form).  Vectors are fine spinors in the layout of
// the context; the odd half of a vector is its second half.
// ---------------------------------------------------------------------------
template <class T>
struct OeBicg {
    dd_ctx* C;
    FineOp<T> op;
    long n, no;          // complex entries of a fine vector and of its odd half
    cx<T>* r; cx<T>* rh; cx<T>* p; cx<T>* v; cx<T>* sv; cx<T>* t; cx<T>* tmp;
    static OeBicg make(dd_ctx* C) {
        OeBicg b;
        b.C = C;
        b.op = fine_op<T>(C);
        b.n = 24L * C->g0.vh;
        b.no = 12L * C->g0.vh;
        const int prec = sizeof(T) == 8 ? 64 : 32;
        if (!C->bicg_ws || C->bicg_prec != prec) {
            C->bicg_ws = C->levels.alloc(sizeof(cx<T>) * 7 * (size_t)b.n);
            C->bicg_prec = prec;
        }
        cx<T>* w = reinterpret_cast<cx<T>*>(C->bicg_ws);
        cx<T>** slot[7] = {&b.r, &b.rh, &b.p, &b.v, &b.sv, &b.t, &b.tmp};
        for (int k = 0; k < 7; k++) *slot[k] = w + (size_t)k * b.n;
        return b;
    }
    cx<T>* odd(cx<T>* a) const { return a + no; }
    // out_o = S x_o  (x, out full vectors; the even half of tmp is used)
    void schur(const cx<T>* x, cx<T>* out) {
        fine_oe_hop<T, T>(op, 0, false, true, 0.0, 1.0, x, x, tmp, C->s);     // tmp_e = A_ee^{-1} D_eo x_o
        fine_oe_hop<T, T>(op, 1, true, false, 1.0, -1.0, x, tmp, out, C->s);  // out_o = A_oo x_o - D_oe tmp_e
    }
    cx<double> dot(const cx<T>* a, const cx<T>* b, int slot) {   // a_o^H b_o into dred[slot]
        vec_multidot<T>(no, 1, a + no, 0, b + no, C->dred + slot, C->dwork, nullptr, C->s);
        return cx<double>{0, 0};
    }
    cx<double> read(int slot) { return C->hred[slot]; }
    // z = (odd-even BiCGStab with `steps` steps) applied to b; returns the steps taken
    int apply(const cx<T>* b, cx<T>* z, int steps) {
        const size_t hb = sizeof(cx<T>) * no;
        // f_o = b_o - D_oe A_ee^{-1} b_e
        fine_oe_hop<T, T>(op, 0, false, true, 1.0, 0.0, b, b, tmp, C->s);       // tmp_e = A_ee^{-1} b_e
        fine_oe_hop<T, T>(op, 1, false, false, 1.0, -1.0, b, tmp, r, C->s);     // r_o = b_o - D_oe tmp_e
        HIPX(hipMemcpyAsync(odd(rh), odd(r), hb, hipMemcpyDeviceToDevice, C->s));
        HIPX(hipMemsetAsync(odd(z), 0, hb, C->s));
        HIPX(hipMemsetAsync(odd(p), 0, hb, C->s));
        HIPX(hipMemsetAsync(odd(v), 0, hb, C->s));
        zc rho_old(1, 0), alpha(1, 0), omega(1, 0);
        int it = 0;
        for (; it < steps; it++) {
            dot(rh, r, 0);
            read_red(C, 1, 1);
            const zc rho(C->hred[0].re, C->hred[0].im);
            if (std::abs(rho) == 0.0) break;
            const zc beta = (rho / rho_old) * (alpha / omega);
            // p = r + beta (p - omega v)
            vec_axpy<T>(no, cx<double>{-omega.real(), -omega.imag()}, odd(v), odd(p), C->s);
            vec_xpay<T>(no, odd(r), cx<double>{beta.real(), beta.imag()}, odd(p), C->s);
            schur(p, v);
            dot(rh, v, 0);
            read_red(C, 1, 1);
            const zc rv(C->hred[0].re, C->hred[0].im);
            if (std::abs(rv) == 0.0) break;
            alpha = rho / rv;
            // s = r - alpha v
            HIPX(hipMemcpyAsync(odd(sv), odd(r), hb, hipMemcpyDeviceToDevice, C->s));
            vec_axpy<T>(no, cx<double>{-alpha.real(), -alpha.imag()}, odd(v), odd(sv), C->s);
            schur(sv, t);
            dot(t, sv, 0);
            dot(t, t, 1);
            read_red(C, 1, 2);
            const zc ts(C->hred[0].re, C->hred[0].im);
            const double tt = C->hred[1].re;
            // x += alpha p (+ omega s)
            vec_axpy<T>(no, cx<double>{alpha.real(), alpha.imag()}, odd(p), odd(z), C->s);
            if (tt == 0.0) { it++; break; }   // s = 0: x is exact
            omega = ts / tt;
            if (std::abs(omega) == 0.0) { it++; break; }   // breakdown: the next beta would divide by omega
            vec_axpy<T>(no, cx<double>{omega.real(), omega.imag()}, odd(sv), odd(z), C->s);
            // r = s - omega t
            HIPX(hipMemcpyAsync(odd(r), odd(sv), hb, hipMemcpyDeviceToDevice, C->s));
            vec_axpy<T>(no, cx<double>{-omega.real(), -omega.imag()}, odd(t), odd(r), C->s);
            rho_old = rho;
        }
        // z_e = A_ee^{-1} (b_e - D_eo z_o)
        fine_oe_hop<T, T>(op, 0, false, true, 1.0, -1.0, b, z, z, C->s);
        return it;
    }
};

template <class T>
struct BicgOps {
    dd_ctx* C;
    OeBicg<T>* B;
    const cx<double>* b;
    cx<double>* x;
    long n;
    int steps;
    cx<T>* Zb;
    cx<double>* V() { return C->oV; }
    cx<T>* Z() { return Zb; }
    cx<T>* vT() { return reinterpret_cast<cx<T>*>(C->ot); }
    cx<double>* t64() { return C->ot + (size_t)C->R * n; }
    void precond(const cx<double>* v, cx<T>* z, const Batch& bt) {
        bvec_convert<T, double>(n, v, vT(), n, bt.nr, bt.mask(), C->s);
        B->apply(vT(), z, steps);
    }
    void matvec(const cx<T>* z, cx<double>* w, const Batch& bt) {
        bvec_convert<double, T>(n, z, t64(), n, bt.nr, bt.mask(), C->s);
        Prof pr(C, DD_K_DIRAC64, 2.0 * C->g0.vh * (144 + 48.0 * bt.count()) * 8);
        fine_dirac<double>(fine_op<double>(C), t64(), w, C->s, bt.nr, n, bt.mask());
    }
    void update(int m, const cx<T>* Z, long ldz, const cx<double>* y, const Batch& bt, const Counts& jc) {
        vec_lincomb<T, double>(n, m, Z, ldz, y, x, C->s, bt.nr, n, 32, n, bt.mask(), &jc);
    }
    void residual(const Batch& bt) {
        fine_dirac<double>(fine_op<double>(C), x, t64(), C->s, bt.nr, n, bt.mask());
        bvec_sub<double>(n, b, t64(), C->oV, n, bt.nr, bt.mask(), C->s);
    }
    std::vector<double> norms(const cx<double>* v, const Batch& bt) { return OuterOps<T>::norms64(C, n, v, bt); }
};

template <class T>
static dd_status bicg_solve_impl(dd_ctx* C, const double* bin, double* xout, double tol, int steps, dd_stats* st) {
    const dd_params& p = C->p;
    const int m = p.outer_restart;
    const long n = 24L * C->g0.vh;
    const long ldv = (long)C->R * n;
    const double t0 = now_s();
    OeBicg<T> B = OeBicg<T>::make(C);
    fine_import_vectors<double>(C->g0, 1, bin, C->ob, C->s);
    HIPX(hipMemsetAsync(C->ox, 0, sizeof(cx<double>) * n, C->s));
    clear_flag(C, DI_BAD);
    vec_finite_check<double>(n, C->ob, C->dflags + DI_BAD, C->s);
    if (read_flag(C, DI_BAD)) fail(DD_ENUMERIC, "NaN/Inf in the right-hand side");
    Batch one{1, C->dflags + DI_ONES, 1u};
    std::vector<double> bn = OuterOps<T>::norms64(C, n, C->ob, one);
    HIPX(hipMemcpyAsync(C->oV, C->ob, sizeof(cx<double>) * n, hipMemcpyDeviceToDevice, C->s));
    BicgOps<T> ops{C, &B, C->ob, C->ox, n, steps, reinterpret_cast<cx<T>*>(C->oV + (size_t)(m + 1) * ldv)};
    KrylovResult res;
    fgmres_batch<double, T>(C, ops, n, ldv, m, tol, p.outer_maxit, 0, one, 0, bn, res);
    fine_export_vectors<double>(C->g0, 1, C->ox, xout, C->s);
    HIPX(hipGetLastError());
    sync(C);
    if (st) {
        memset(st, 0, sizeof *st);
        st->outer_iters = (int)res.its[0];
        st->restarts = res.restarts[0];
        st->coarse_iters[0] = (long)res.its[0] * steps;   // BiCGStab steps (each two S applies)
        st->true_relres = res.relres[0];
        st->converged = res.conv[0] ? 1 : 0;
        st->solve_s = now_s() - t0;
    }
    return res.conv[0] ? DD_OK : DD_ENOCONV;
}


// ---------------------------------------------------------------------------
// Comparison solver of Sec. 4.1: inexact deflation, FP64, two levels.
//   pi_R v = v - P D_c^{-1} P^H D v, every D_c^{-1} the coarsest odd-even GMRES
//   run to relative residual ctol;
//   chi' = P D_c^{-1} P^H b;  FGMRES on D pi_R chi = b - D chi' right-
//   preconditioned by nu SAP iterations from zero;  x = pi_R chi + chi'.
// ---------------------------------------------------------------------------
struct IdDefl {
    dd_ctx* C;
    Hier<double>* H;
    long n;
    double ctol;
    cx<double>* b0; cx<double>* chi1; cx<double>* t1; cx<double>* t2; cx<double>* t3;
    static IdDefl make(dd_ctx* C, Hier<double>* H, double ctol) {
        IdDefl d;
        d.C = C;
        d.H = H;
        d.n = 24L * C->g0.vh;
        d.ctol = ctol;
        if (!C->id_ws) C->id_ws = C->levels.alloc(sizeof(cx<double>) * 5 * (size_t)d.n);
        cx<double>* w = reinterpret_cast<cx<double>*>(C->id_ws);
        cx<double>** slot[5] = {&d.b0, &d.chi1, &d.t1, &d.t2, &d.t3};
        for (int k = 0; k < 5; k++) *slot[k] = w + (size_t)k * d.n;
        return d;
    }
    // out = P D_c^{-1} P^H in
    void coarse_correction(const cx<double>* in, cx<double>* out, const Batch& bt) {
        H->restrict_(0, in, H->rc[1], bt);
        const double keep = C->p.coarse_tol;
        C->p.coarse_tol = ctol;
        try {
            H->gmres_oe(1, H->rc[1], H->ec[1], bt);
        } catch (...) {
            C->p.coarse_tol = keep;
            throw;
        }
        C->p.coarse_tol = keep;
        H->prolong(0, H->ec[1], out, bt);
    }
    void dirac(const cx<double>* in, cx<double>* out, const Batch& bt) {
        Prof pr(C, DD_K_DIRAC64, 2.0 * C->g0.vh * (144 + 48.0 * bt.count()) * 8);
        fine_dirac<double>(fine_op<double>(C), in, out, C->s, bt.nr, n, bt.mask());
    }
    // out = pi_R in (out distinct from in; t1, t2 are used)
    void pi_R(const cx<double>* in, cx<double>* out, const Batch& bt) {
        dirac(in, t1, bt);
        coarse_correction(t1, t2, bt);
        bvec_sub<double>(n, in, t2, out, n, bt.nr, bt.mask(), C->s);
    }
    // out = D pi_R in (t1, t2, t3 are used)
    void deflated(const cx<double>* in, cx<double>* out, const Batch& bt) {
        pi_R(in, t3, bt);
        dirac(t3, out, bt);
    }
};

struct IdOps {
    dd_ctx* C;
    IdDefl* Dp;
    const cx<double>* b;
    cx<double>* x;
    long n;
    int nu;
    cx<double>* Zb;
    cx<double>* V() { return C->oV; }
    cx<double>* Z() { return Zb; }
    void precond(const cx<double>* v, cx<double>* z, const Batch& bt) { Dp->H->sap(0, v, z, nu, true, bt); }
    void matvec(const cx<double>* z, cx<double>* w, const Batch& bt) { Dp->deflated(z, w, bt); }
    void update(int m, const cx<double>* Z, long ldz, const cx<double>* y, const Batch& bt, const Counts& jc) {
        vec_lincomb<double, double>(n, m, Z, ldz, y, x, C->s, bt.nr, n, 32, n, bt.mask(), &jc);
    }
    void residual(const Batch& bt) {
        Dp->deflated(x, Dp->t1, bt);
        bvec_sub<double>(n, b, Dp->t1, C->oV, n, bt.nr, bt.mask(), C->s);
    }
    std::vector<double> norms(const cx<double>* v, const Batch& bt) { return OuterOps<double>::norms64(C, n, v, bt); }
};

static dd_status id_solve_impl(dd_ctx* C, Hier<double>& H, const double* bin, double* xout, double tol, int nu,
                               double ctol, dd_stats* st) {
    const dd_params& p = C->p;
    const int m = p.outer_restart;
    const long n = 24L * C->g0.vh;
    const long ldv = (long)C->R * n;
    const double t0 = now_s();
    IdDefl Dp = IdDefl::make(C, &H, ctol);
    Batch one{1, C->dflags + DI_ONES, 1u};
    fine_import_vectors<double>(C->g0, 1, bin, Dp.b0, C->s);
    clear_flag(C, DI_BAD);
    vec_finite_check<double>(n, Dp.b0, C->dflags + DI_BAD, C->s);
    if (read_flag(C, DI_BAD)) fail(DD_ENUMERIC, "NaN/Inf in the right-hand side");
    memset(H.coarse_count, 0, sizeof H.coarse_count);
    // chi' = P D_c^{-1} P^H b and the deflated right-hand side pi_L b = b - D chi'
    Dp.coarse_correction(Dp.b0, Dp.chi1, one);
    Dp.dirac(Dp.chi1, Dp.t1, one);
    bvec_sub<double>(n, Dp.b0, Dp.t1, C->ob, n, 1, one.mask(), C->s);
    HIPX(hipMemsetAsync(C->ox, 0, sizeof(cx<double>) * n, C->s));
    std::vector<double> bn = OuterOps<double>::norms64(C, n, C->ob, one);
    HIPX(hipMemcpyAsync(C->oV, C->ob, sizeof(cx<double>) * n, hipMemcpyDeviceToDevice, C->s));
    IdOps ops{C, &Dp, C->ob, C->ox, n, nu, C->oV + (size_t)(m + 1) * ldv};
    KrylovResult res;
    fgmres_batch<double, double>(C, ops, n, ldv, m, tol, p.outer_maxit, 0, one, 0, bn, res);
    // x = pi_R chi + chi'
    Dp.pi_R(C->ox, Dp.t3, one);
    vec_axpy<double>(n, cx<double>{1.0, 0.0}, Dp.chi1, Dp.t3, C->s);
    // its true residual
    Dp.dirac(Dp.t3, Dp.t1, one);
    bvec_sub<double>(n, Dp.b0, Dp.t1, Dp.t2, n, 1, one.mask(), C->s);
    const double rn = OuterOps<double>::norms64(C, n, Dp.t2, one)[0];
    const double b0n = OuterOps<double>::norms64(C, n, Dp.b0, one)[0];
    fine_export_vectors<double>(C->g0, 1, Dp.t3, xout, C->s);
    HIPX(hipGetLastError());
    sync(C);
    if (st) {
        memset(st, 0, sizeof *st);
        st->outer_iters = (int)res.its[0];
        st->restarts = res.restarts[0];
        st->coarse_iters[1] = H.coarse_count[1][0];
        st->true_relres = b0n > 0 ? rn / b0n : 0.0;
        st->converged = res.conv[0] ? 1 : 0;
        st->solve_s = now_s() - t0;
    }
    return res.conv[0] ? DD_OK : DD_ENOCONV;
}

// ---------------------------------------------------------------------------
// Fixed staging memory of the allocation-free stencil entry point
// (dd_apply_D_noalloc): the two internal-layout FP64 spinors that dd_apply
// allocates per call live here instead.  Every GPU the library runs on holds
// its own copy until the process ends; host code uses the address that
// hipGetSymbolAddress returns for the current device, never the array's name.
// ---------------------------------------------------------------------------
static const size_t NOALLOC_SITES = 65536;                        // a 16^4 lattice
static const size_t NOALLOC_BYTES = NOALLOC_SITES * 2 * 12 * 16;  // two FP64 spinors: 24 MiB
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

static const int NOALLOC_MAXDEV = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAXDEV];

// address of `scratch` on the current device, looked up once per device
static void* scratch_for_current_device() {
    int dev = -1;
    HIPX(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAXDEV) fail(DD_EDEVICE, "device index " + std::to_string(dev) + " out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(DD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
static std::string g_create_error;

#define ABI_TRY(ctx)                    \
    if (!(ctx)) return DD_EINVAL;       \
    try {
#define ABI_END(ctx)                                  \
    }                                                 \
    catch (const DdError& e) {                        \
        (ctx)->err = e.msg;                           \
        return e.code;                                \
    }                                                 \
    catch (const std::exception& e) {                 \
        (ctx)->err = e.what();                        \
        return DD_EDEVICE;                            \
    }

// The public functions below were declared with C linkage in ddamg.h.

void dd_default_params(dd_params* p) {
    memset(p, 0, sizeof *p);
    p->levels = 2;
    for (int l = 0; l < DD_MAXLEV; l++) {
        p->n_tv[l] = 20;
        p->mr_steps[l] = 4;
        for (int mu = 0; mu < 4; mu++) {
            p->agg[l][mu] = (l == 0) ? 4 : 2;
            p->sap[l][mu] = (l == 0) ? 4 : 2;
        }
    }
    p->nu = 2;
    p->n_inv = 6;
    p->coarse_tol = 5e-2;
    p->coarse_restart = 30;
    p->coarse_maxit = 1000;
    p->coarse_fixed = 0;
    p->mid_tol = 5e-2;
    p->mid_restart = 10;
    p->mid_maxit = 50;
    p->mid_fixed = 0;
    p->outer_restart = 25;
    p->outer_maxit = 2000;
    p->precision = 64;
    p->given_vectors = 0;
    p->seed = 0x5eedULL;
    p->max_rhs = 1;
}

const char* dd_last_error(const dd_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

dd_status dd_create(dd_ctx** out, const int dims[4], const double* gauge, const double* clover, double m0, double csw,
                    void* hip_stream) {
    if (!out || !dims || !gauge) {
        g_create_error = "dd_create: NULL argument";
        return DD_EINVAL;
    }
    *out = nullptr;
    for (int mu = 0; mu < 4; mu++)
        if (dims[mu] < 2 || (dims[mu] & 1)) {
            g_create_error = "dd_create: lattice extents must be even and >= 2";
            return DD_EINVAL;
        }
    dd_ctx* C = new dd_ctx();
    try {
        C->s = (hipStream_t)hip_stream;
        HIPX(hipStreamCreateWithFlags(&C->cap, hipStreamNonBlocking));
        memcpy(C->dims, dims, sizeof(int) * 4);
        C->vol = (long)dims[0] * dims[1] * dims[2] * dims[3];
        if (C->vol / 2 > 0x7fffffffL / 24) fail(DD_EINVAL, "lattice too large");
        C->m0 = m0;
        C->csw = csw;
        HIPX(hipHostMalloc((void**)&C->hred, sizeof(cx<double>) * MAX_RHS * RS, hipHostMallocDefault));
        HIPX(hipHostMalloc((void**)&C->hy, sizeof(cx<double>) * MAX_RHS * 32, hipHostMallocDefault));
        HIPX(hipHostMalloc((void**)&C->hint, sizeof(int) * DI_WORDS, hipHostMallocDefault));
        int b[4];
        bool four = true;
        for (int mu = 0; mu < 4; mu++) { b[mu] = 4; if (dims[mu] % 4 || ((dims[mu] / 4) != 1 && ((dims[mu] / 4) & 1))) four = false; }
        if (!four) for (int mu = 0; mu < 4; mu++) b[mu] = 2;
        if (!valid_layout(dims, b, true)) fail(DD_EINVAL, "lattice extents admit no 2-colourable block layout");
        layout_fields(C, b, gauge, clover);
        dd_default_params(&C->p);
        try {
            C->scratch = scratch_for_current_device();
        } catch (const DdError& e) {
            C->scratch_err = e.msg;   // only dd_apply_D_noalloc needs it; it reports this
        }
    } catch (const DdError& e) {
        g_create_error = e.msg;
        delete C;
        return e.code;
    }
    *out = C;
    return DD_OK;
}

void dd_destroy(dd_ctx* ctx) { delete ctx; }

static void configure_impl(dd_ctx* C, const dd_params* pin) {
    dd_params p = *pin;
    if (p.levels < 2 || p.levels > DD_MAXLEV) fail(DD_EINVAL, "levels must be 2 .. " + std::to_string(DD_MAXLEV));
    if (p.precision != 64 && p.precision != 32 && p.precision != 16) fail(DD_EINVAL, "precision must be 64, 32 or 16");
    if (p.outer_restart < 1 || p.outer_restart > 32 || p.coarse_restart < 1 || p.coarse_restart > 32 || p.mid_restart < 1 ||
        p.mid_restart > 32)
        fail(DD_EINVAL, "restart lengths must be in 1..32");
    if (p.nu < 0 || p.n_inv < 0) fail(DD_EINVAL, "nu and n_inv must be >= 0");
    if (p.max_rhs < 1 || p.max_rhs > MAX_RHS) fail(DD_EINVAL, "max_rhs must be in 1.." + std::to_string(MAX_RHS));
    if (!valid_layout(C->dims, p.sap[0], true))
        fail(DD_EINVAL, "SAP blocks must be powers of two dividing the lattice with an even block count (or 1) per dimension");
    if (p.sap[0][0] * p.sap[0][1] * p.sap[0][2] * p.sap[0][3] > 256) fail(DD_EINVAL, "fine SAP blocks hold at most 256 sites");
    C->H64.reset();
    C->H32.reset();
    C->levels.release();
    C->configured = false;
    C->have_setup = false;
    C->stream = dd_ctx::StreamSlots{};
    C->bicg_ws = nullptr;
    C->bicg_prec = 0;
    C->id_ws = nullptr;
    C->p = p;
    // re-layout the fine fields if the SAP blocks differ from the current layout
    bool same = true;
    for (int mu = 0; mu < 4; mu++) same = same && (C->g0.b[mu] == p.sap[0][mu]);
    if (!same) layout_fields(C, p.sap[0], C->gauge_canon, C->clover_canon);
    {
        int dev = 0, maxlds = 0, a = 0;
        HIPX(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&a, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess) maxlds = std::max(maxlds, a);
        if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) maxlds = std::max(maxlds, a);
        if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess)
            maxlds = std::max(maxlds, a);
        (void)hipGetLastError();
        size_t need = (p.precision == 64) ? fine_sap_lds_bytes<double>(C->g0) : fine_sap_lds_bytes<float>(C->g0);
        if (need > (size_t)maxlds)
            fail(DD_EINVAL, "SAP blocks need " + std::to_string(need) + " bytes of LDS per workgroup at this precision; the "
                            "device offers " + std::to_string(maxlds));
    }
    // FP64 outer workspace for R = max_rhs right-hand sides: V (m+1 sets),
    // Z (m sets, preconditioner precision), b, x and two temporary sets
    C->R = p.max_rhs;
    const size_t nR = (size_t)24 * C->g0.vh * C->R;
    size_t zbytes = (p.precision == 64) ? sizeof(cx<double>) : sizeof(cx<float>);
    size_t vbytes = sizeof(cx<double>) * (size_t)(p.outer_restart + 1) * nR + zbytes * (size_t)p.outer_restart * nR;
    C->oV = reinterpret_cast<cx<double>*>(C->levels.alloc(vbytes));
    C->ot = C->levels.get<cx<double>>(2 * nR);
    C->ob = C->levels.get<cx<double>>(nR);
    C->ox = C->levels.get<cx<double>>(nR);
    if (p.precision == 64) {
        C->H64.reset(new Hier<double>(C));
        C->H64->build_geometry();
    } else {
        C->H32.reset(new Hier<float>(C));
        C->H32->build_geometry();
    }
    C->configured = true;
}

dd_status dd_configure(dd_ctx* ctx, const dd_params* p) {
    ABI_TRY(ctx)
    dd_params d;
    if (!p) { dd_default_params(&d); p = &d; }
    configure_impl(ctx, p);
    return DD_OK;
    ABI_END(ctx)
}

template <class T>
static void setup_all(dd_ctx* C, Hier<T>& H) {
    for (int l = 0; l + 1 < H.nlev; l++) H.setup_level(l, C->p.given_vectors != 0);
}

dd_status dd_setup(dd_ctx* ctx, int n_tv, const int block[4], int levels, const dd_params* pin) {
    ABI_TRY(ctx)
    double t0 = now_s();
    dd_params p;
    if (pin) p = *pin;
    else dd_default_params(&p);
    if (n_tv > 0) p.n_tv[0] = n_tv;
    if (levels > 0) p.levels = levels;
    if (block)
        for (int mu = 0; mu < 4; mu++) p.agg[0][mu] = p.sap[0][mu] = block[mu];
    // given_vectors: the hierarchy was configured (dd_configure) and the initial
    // test vectors installed (dd_set_test_vectors); its parameters are used as is
    if (p.given_vectors) {
        if (!ctx->configured) fail(DD_ESTATE, "given_vectors requires dd_configure + dd_set_test_vectors first");
        ctx->p.given_vectors = 1;
    } else {
        configure_impl(ctx, &p);
    }
    if (ctx->H64) setup_all(ctx, *ctx->H64);
    else setup_all(ctx, *ctx->H32);
    sync(ctx);
    ctx->have_setup = true;
    ctx->last_setup_s = now_s() - t0;
    return DD_OK;
    ABI_END(ctx)
}

// k right-hand sides (device, canonical layout) solved in batches of at most R
template <class T>
static dd_status solve_impl(dd_ctx* C, Hier<T>& H, int k, const double* b, double* x, double tol, dd_stats* st) {
    const long n = 24L * C->g0.vh;
    const size_t canon = (size_t)24 * C->vol;
    dd_status worst = DD_OK;
    for (int q0 = 0; q0 < k; q0 += C->R) {
        const int nr = std::min(C->R, k - q0);
        const double t0 = now_s();
        fine_import_vectors<double>(C->g0, nr, b + q0 * canon, C->ob, C->s);
        dd_status rc[MAX_RHS];
        dd_stats sb[MAX_RHS];
        memset(sb, 0, sizeof sb);
        outer_fgmres<T>(C, H, nr, tol, 0, sb, rc);
        fine_export_vectors<double>(C->g0, nr, C->ox, x + q0 * canon, C->s);
        HIPX(hipGetLastError());
        sync(C);
        const double dt = now_s() - t0;
        (void)n;
        for (int r = 0; r < nr; r++) {
            sb[r].solve_s = dt;
            sb[r].setup_s = C->last_setup_s;
            if (st) st[q0 + r] = sb[r];
            if (rc[r] != DD_OK && worst == DD_OK) worst = rc[r];
        }
    }
    return worst;
}

dd_status dd_solve(dd_ctx* ctx, const double* b, double* x, double tol, dd_stats* st) {
    ABI_TRY(ctx)
    if (!ctx->have_setup) fail(DD_ESTATE, "dd_solve before dd_setup");
    if (ctx->stream.any()) fail(DD_ESTATE, "dd_solve while continuous-batching slots are in use");
    if (!b || !x) fail(DD_EINVAL, "NULL vector");
    if (!(tol > 0)) fail(DD_EINVAL, "tol must be positive");
    dd_status rc = ctx->H64 ? solve_impl(ctx, *ctx->H64, 1, b, x, tol, st) : solve_impl(ctx, *ctx->H32, 1, b, x, tol, st);
    if (rc == DD_ENOCONV) ctx->err = "outer FGMRES reached outer_maxit";
    return rc;
    ABI_END(ctx)
}

dd_status dd_solve_batch(dd_ctx* ctx, int k, const double* b, double* x, double tol, dd_stats* st) {
    ABI_TRY(ctx)
    if (k < 0) fail(DD_EINVAL, "k < 0");
    if (k == 0) return DD_OK;
    if (!ctx->have_setup) fail(DD_ESTATE, "dd_solve_batch before dd_setup");
    if (ctx->stream.any()) fail(DD_ESTATE, "dd_solve_batch while continuous-batching slots are in use");
    if (!b || !x) fail(DD_EINVAL, "NULL vector");
    if (!(tol > 0)) fail(DD_EINVAL, "tol must be positive");
    dd_status rc = ctx->H64 ? solve_impl(ctx, *ctx->H64, k, b, x, tol, st) : solve_impl(ctx, *ctx->H32, k, b, x, tol, st);
    if (rc == DD_ENOCONV) ctx->err = "outer FGMRES reached outer_maxit for at least one right-hand side";
    return rc;
    ABI_END(ctx)
}

dd_status dd_solve_bicgstab(dd_ctx* ctx, const double* b, double* x, double tol, int steps, int precision,
                            dd_stats* st) {
    ABI_TRY(ctx)
    if (!ctx->configured) fail(DD_ESTATE, "dd_solve_bicgstab needs dd_configure (outer workspace)");
    if (ctx->stream.any()) fail(DD_ESTATE, "dd_solve_bicgstab while continuous-batching slots are in use");
    if (!b || !x) fail(DD_EINVAL, "NULL vector");
    if (!(tol > 0) || steps < 1) fail(DD_EINVAL, "tol must be positive and steps >= 1");
    if (precision != 32 && precision != 64) fail(DD_EINVAL, "precision must be 32 or 64");
    dd_status rc = (precision == 64) ? bicg_solve_impl<double>(ctx, b, x, tol, steps, st)
                                     : bicg_solve_impl<float>(ctx, b, x, tol, steps, st);
    if (rc == DD_ENOCONV) ctx->err = "outer FGMRES reached outer_maxit";
    return rc;
    ABI_END(ctx)
}

dd_status dd_solve_id(dd_ctx* ctx, const double* b, double* x, double tol, int nu, double coarse_tol, dd_stats* st) {
    ABI_TRY(ctx)
    if (!ctx->have_setup) fail(DD_ESTATE, "dd_solve_id before dd_setup");
    if (!ctx->H64 || ctx->H64->nlev != 2) fail(DD_ESTATE, "inexact deflation runs on an FP64 two-level setup");
    if (ctx->stream.any()) fail(DD_ESTATE, "dd_solve_id while continuous-batching slots are in use");
    if (!b || !x) fail(DD_EINVAL, "NULL vector");
    if (!(tol > 0) || !(coarse_tol > 0) || nu < 1) fail(DD_EINVAL, "tolerances must be positive and nu >= 1");
    dd_status rc = id_solve_impl(ctx, *ctx->H64, b, x, tol, nu, coarse_tol, st);
    if (rc == DD_ENOCONV) ctx->err = "outer FGMRES reached outer_maxit";
    return rc;
    ABI_END(ctx)
}

// ---------------------------------------------------------------------------
// continuous batching: slots of the outer FGMRES loaded, cycled and read out
// one restart cycle at a time
// ---------------------------------------------------------------------------
template <class T>
static void stream_load_impl(dd_ctx* C, Hier<T>& H, int slot, const double* b, double tol) {
    auto& S = C->stream;
    const long n = 24L * C->g0.vh;
    if ((int)S.hs.size() != C->R) S.hs.assign(C->R, Hess(C->p.outer_restart));
    fine_import_vectors<double>(C->g0, 1, b, C->ob + (size_t)slot * n, C->s);
    clear_flag(C, DI_BAD);
    vec_finite_check<double>(n, C->ob + (size_t)slot * n, C->dflags + DI_BAD, C->s);
    if (read_flag(C, DI_BAD)) fail(DD_ENUMERIC, "NaN/Inf in the right-hand side");
    HIPX(hipMemsetAsync(C->ox + (size_t)slot * n, 0, sizeof(cx<double>) * n, C->s));
    HIPX(hipMemcpyAsync(C->oV + (size_t)slot * n, C->ob + (size_t)slot * n, sizeof(cx<double>) * n,
                        hipMemcpyDeviceToDevice, C->s));
    // no cycle is running: the outer FGMRES's own mask words carry this slot
    Batch all{C->R, C->dflags + DI_ONES, (C->R >= 32) ? ~0u : ((1u << C->R) - 1)};
    Batch one = with_mask(C, all, 0, 1u << slot);
    std::vector<double> nb = OuterOps<T>::norms64(C, n, C->ob, one);
    S.bnorm[slot] = S.beta[slot] = nb[slot];
    S.tol[slot] = tol;
    S.its[slot] = 0;
    S.restarts[slot] = 0;
    for (int l = 0; l < DD_MAXLEV; l++) H.coarse_count[l][slot] = 0;
    S.state[slot] = (nb[slot] == 0) ? DD_SLOT_CONVERGED : DD_SLOT_RUNNING;
}

static void stream_stats(dd_ctx* C, int r, dd_stats* st, const long (*cc)[MAX_RHS]) {
    auto& S = C->stream;
    memset(st, 0, sizeof *st);
    st->outer_iters = (int)S.its[r];
    st->restarts = S.restarts[r];
    for (int l = 0; l < DD_MAXLEV; l++) st->coarse_iters[l] = cc[l][r];
    st->true_relres = S.bnorm[r] > 0 ? S.beta[r] / S.bnorm[r] : 0.0;
    st->converged = S.state[r] == DD_SLOT_CONVERGED;
    st->setup_s = C->last_setup_s;
}

template <class T>
static void stream_cycle_impl(dd_ctx* C, Hier<T>& H, int* state, dd_stats* st) {
    auto& S = C->stream;
    const dd_params& p = C->p;
    const int m = p.outer_restart, R = C->R;
    const long n = 24L * C->g0.vh, ldv = (long)R * n;
    unsigned cyc = 0;
    for (int r = 0; r < R; r++) {
        if (S.state[r] != DD_SLOT_RUNNING) continue;
        if (S.beta[r] <= S.tol[r] * S.bnorm[r]) S.state[r] = DD_SLOT_CONVERGED;
        else if (S.its[r] >= p.outer_maxit) S.state[r] = DD_SLOT_STOPPED;
        else cyc |= 1u << r;
    }
    if (cyc) {
        const double t0 = now_s();
        Batch all{R, C->dflags + DI_ONES, (R >= 32) ? ~0u : ((1u << R) - 1)};
        with_outer_ops(C, H, [&](auto& ops, auto* zs) {
            using ZS = std::remove_pointer_t<decltype(zs)>;
            fgmres_cycle<double, ZS>(C, ops, n, ldv, m, S.tol, p.outer_maxit, 0, all, 0, cyc, S.hs, S.beta, S.bnorm,
                                     S.its);
        });
        sync(C);
        (void)t0;
        for (int r = 0; r < R; r++) {
            if (!((cyc >> r) & 1u)) continue;
            if (S.beta[r] <= S.tol[r] * S.bnorm[r]) S.state[r] = DD_SLOT_CONVERGED;
            else if (S.its[r] >= p.outer_maxit) S.state[r] = DD_SLOT_STOPPED;
            else S.restarts[r]++;
        }
    }
    for (int r = 0; r < R; r++) {
        if (state) state[r] = S.state[r];
        if (st) stream_stats(C, r, st + r, H.coarse_count);
    }
}

dd_status dd_stream_load(dd_ctx* ctx, int slot, const double* b, double tol) {
    ABI_TRY(ctx)
    if (!ctx->have_setup) fail(DD_ESTATE, "dd_stream_load before dd_setup");
    if (slot < 0 || slot >= ctx->R) fail(DD_EINVAL, "slot out of range 0..max_rhs-1");
    if (ctx->stream.state[slot] != DD_SLOT_FREE) fail(DD_ESTATE, "slot in use");
    if (!b) fail(DD_EINVAL, "NULL vector");
    if (!(tol > 0)) fail(DD_EINVAL, "tol must be positive");
    if (ctx->H64) stream_load_impl(ctx, *ctx->H64, slot, b, tol);
    else stream_load_impl(ctx, *ctx->H32, slot, b, tol);
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_stream_cycle(dd_ctx* ctx, int* state, dd_stats* st) {
    ABI_TRY(ctx)
    if (!ctx->have_setup) fail(DD_ESTATE, "dd_stream_cycle before dd_setup");
    if (ctx->H64) stream_cycle_impl(ctx, *ctx->H64, state, st);
    else stream_cycle_impl(ctx, *ctx->H32, state, st);
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_stream_take(dd_ctx* ctx, int slot, double* x, dd_stats* st) {
    ABI_TRY(ctx)
    if (slot < 0 || slot >= ctx->R) fail(DD_EINVAL, "slot out of range 0..max_rhs-1");
    auto& S = ctx->stream;
    if (S.state[slot] != DD_SLOT_CONVERGED && S.state[slot] != DD_SLOT_STOPPED) fail(DD_ESTATE, "slot not finished");
    if (!x) fail(DD_EINVAL, "NULL vector");
    const long n = 24L * ctx->g0.vh;
    fine_export_vectors<double>(ctx->g0, 1, ctx->ox + (size_t)slot * n, x, ctx->s);
    HIPX(hipGetLastError());
    sync(ctx);
    if (st) {
        if (ctx->H64) stream_stats(ctx, slot, st, ctx->H64->coarse_count);
        else stream_stats(ctx, slot, st, ctx->H32->coarse_count);
    }
    const bool ok = S.state[slot] == DD_SLOT_CONVERGED;
    S.state[slot] = DD_SLOT_FREE;
    if (!ok) fail(DD_ENOCONV, "the right-hand side of this slot reached outer_maxit");
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_set_mass(dd_ctx* ctx, double m0) {
    ABI_TRY(ctx)
    for (int r = 0; r < MAX_RHS; r++)
        if (ctx->stream.state[r] == DD_SLOT_RUNNING) fail(DD_ESTATE, "dd_set_mass while continuous-batching slots run");
    double dm = m0 - ctx->m0;
    clear_flag(ctx, DI_BAD);
    fine_clover_shift(ctx->g0, dm, ctx->clov64, ctx->clovinv64, ctx->dflags + DI_BAD, ctx->s);
    vec_convert<float, double>((long)ctx->vol * 36, reinterpret_cast<const cx<double>*>(ctx->clov64),
                               reinterpret_cast<cx<float>*>(ctx->clov32), ctx->s);
    vec_convert<float, double>((long)ctx->vol * 36, reinterpret_cast<const cx<double>*>(ctx->clovinv64),
                               reinterpret_cast<cx<float>*>(ctx->clovinv32), ctx->s);
    if (read_flag(ctx, DI_BAD)) fail(DD_ENUMERIC, "singular clover block after the mass shift");
    ctx->m0 = m0;
    auto shift = [&](auto& H) {
        for (int l = 1; l < H.nlev; l++) {
            coarse_shift_diag(H.g[l], H.nd[l], dm, H.M[l], ctx->s);
            coarse_self_inverse(H.g[l], H.nd[l], H.M[l], H.Minv[l], ctx->dflags + DI_BAD, ctx->s);
            H.fold(l);
            H.refresh_half(l - 1);
        }
        if (H.half) {
            const long vol = 2L * H.g[0].vh;
            vec_convert<_Float16, float>(vol * 36, reinterpret_cast<const cx<float>*>(ctx->clov32),
                                         reinterpret_cast<cx<_Float16>*>(ctx->clov16), ctx->s);
            vec_convert<_Float16, float>(vol * 36, reinterpret_cast<const cx<float>*>(ctx->clovinv32),
                                         reinterpret_cast<cx<_Float16>*>(ctx->clovinv16), ctx->s);
        }
    };
    if (ctx->configured) {
        if (ctx->H64) shift(*ctx->H64);
        else shift(*ctx->H32);
        if (read_flag(ctx, DI_BAD)) fail(DD_ENUMERIC, "singular coarse self block after the mass shift");
    }
    return DD_OK;
    ABI_END(ctx)
}

template <class T>
static void set_vectors_impl(dd_ctx* C, Hier<T>& H, int l, int n, const double* v) {
    if (l < 0 || l >= H.nlev - 1) fail(DD_EINVAL, "no transfer on this level");
    if (n != H.N[l]) fail(DD_EINVAL, "vector count differs from n_tv of the level");
    if (l == 0) fine_import_vectors<T>(H.g[0], n, v, H.tv[0], C->s);
    else coarse_import_vector<T>(H.g[l], H.nd[l], n, v, H.tv[l], C->s);
    sync(C);
}

dd_status dd_set_test_vectors(dd_ctx* ctx, int level, int n, const double* v) {
    ABI_TRY(ctx)
    if (!ctx->configured) fail(DD_ESTATE, "dd_configure first");
    if (ctx->H64) set_vectors_impl(ctx, *ctx->H64, level, n, v);
    else set_vectors_impl(ctx, *ctx->H32, level, n, v);
    return DD_OK;
    ABI_END(ctx)
}

template <class T>
static void get_vectors_impl(dd_ctx* C, Hier<T>& H, int l, double* v, bool P) {
    if (l < 0 || l >= H.nlev - 1) fail(DD_EINVAL, "no transfer on this level");
    const cx<T>* src = P ? H.P[l] : H.tv[l];
    if (l == 0) fine_export_vectors<T>(H.g[0], H.N[0], src, v, C->s);
    else coarse_export_vector<T>(H.g[l], H.nd[l], H.N[l], src, v, C->s);
    sync(C);
}

dd_status dd_get_test_vectors(dd_ctx* ctx, int level, double* v) {
    ABI_TRY(ctx)
    if (!ctx->configured) fail(DD_ESTATE, "not configured");
    if (ctx->H64) get_vectors_impl(ctx, *ctx->H64, level, v, false);
    else get_vectors_impl(ctx, *ctx->H32, level, v, false);
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_get_P(dd_ctx* ctx, int level, double* out) {
    ABI_TRY(ctx)
    if (!ctx->configured) fail(DD_ESTATE, "not configured");
    if (ctx->H64) get_vectors_impl(ctx, *ctx->H64, level, out, true);
    else get_vectors_impl(ctx, *ctx->H32, level, out, true);
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_build_level(dd_ctx* ctx, int level) {
    ABI_TRY(ctx)
    if (!ctx->configured) fail(DD_ESTATE, "dd_configure first");
    auto go = [&](auto& H) {
        if (level < 0 || level >= H.nlev - 1) fail(DD_EINVAL, "no transfer on this level");
        H.build(level);
    };
    if (ctx->H64) go(*ctx->H64);
    else go(*ctx->H32);
    sync(ctx);
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_mark_setup(dd_ctx* ctx) {
    ABI_TRY(ctx)
    if (!ctx->configured) fail(DD_ESTATE, "dd_configure first");
    ctx->have_setup = true;
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_get_coarse(dd_ctx* ctx, int level, double* Mout, double* Minvout) {
    ABI_TRY(ctx)
    if (!ctx->configured) fail(DD_ESTATE, "not configured");
    auto go = [&](auto& H) {
        if (level < 1 || level >= H.nlev) fail(DD_EINVAL, "no coarse operator on this level");
        if (Mout) coarse_export_blocks(H.g[level], H.nd[level], 9, H.M[level], Mout, ctx->s);
        if (Minvout) coarse_export_blocks(H.g[level], H.nd[level], 1, H.Minv[level], Minvout, ctx->s);
    };
    if (ctx->H64) go(*ctx->H64);
    else go(*ctx->H32);
    sync(ctx);
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_get_clover(dd_ctx* ctx, double* A, double* Ainv) {
    ABI_TRY(ctx)
    if (A) fine_clover_export(ctx->g0, ctx->clov64, A, ctx->s);
    if (Ainv) fine_clover_export(ctx->g0, ctx->clovinv64, Ainv, ctx->s);
    sync(ctx);
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_level_info(const dd_ctx* ctx, int level, int dims[4], int* nd) {
    if (!ctx) return DD_EINVAL;
    if (level == 0) {
        memcpy(dims, ctx->dims, sizeof(int) * 4);
        *nd = 12;
        return DD_OK;
    }
    const Geom* g = nullptr;
    int n = 0;
    if (ctx->H64 && level < ctx->H64->nlev) { g = &ctx->H64->g[level]; n = ctx->H64->nd[level]; }
    if (ctx->H32 && level < ctx->H32->nlev) { g = &ctx->H32->g[level]; n = ctx->H32->nd[level]; }
    if (!g) return DD_EINVAL;
    memcpy(dims, g->d, sizeof(int) * 4);
    *nd = n;
    return DD_OK;
}

dd_status dd_profile_classes(dd_ctx* ctx, unsigned class_mask) {
    ABI_TRY(ctx)
    if (class_mask >> DD_K_NCLASS) fail(DD_EINVAL, "class mask names an unknown kernel class");
    sync(ctx);
    ctx->prof_mask = class_mask;
    ctx->prof_on = class_mask != 0;
    if (class_mask) {
        for (int k = 0; k < DD_K_NCLASS; k++) { ctx->prof_n[k] = 0; ctx->prof_ms[k] = 0; ctx->prof_bytes[k] = 0; }
    }
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_profile(dd_ctx* ctx, int enable) {
    return dd_profile_classes(ctx, enable ? (1u << DD_K_NCLASS) - 1u : 0u);
}

dd_status dd_profile_read(dd_ctx* ctx, int cls, long* launches, double* total_ms, double* total_bytes) {
    ABI_TRY(ctx)
    if (cls < 0 || cls >= DD_K_NCLASS) fail(DD_EINVAL, "unknown kernel class");
    sync(ctx);
    if (launches) *launches = ctx->prof_n[cls];
    if (total_ms) *total_ms = ctx->prof_ms[cls];
    if (total_bytes) *total_bytes = ctx->prof_bytes[cls];
    return DD_OK;
    ABI_END(ctx)
}

template <class T>
static double time_prec(dd_ctx* C, Hier<T>& H, int cls, int reps) {
    const long n = 24L * C->g0.vh;
    fine_random<T>(H.g[0], 1, 12345ULL, 7, H.wa[0], C->s);
    HIPX(hipMemsetAsync(H.wb[0], 0, sizeof(cx<T>) * n, C->s));
    hipEvent_t a = ev_get(C), b = ev_get(C);
    // one untimed launch first
    if (cls == DD_K_DIRAC_PREC) H.apply_D(0, H.wa[0], H.wb[0], single(C));
    else H.sap(0, H.wa[0], H.wb[0], 1, false, single(C));
    HIPX(hipEventRecord(a, C->s));
    for (int r = 0; r < reps; r++) {
        if (cls == DD_K_DIRAC_PREC) H.apply_D(0, H.wa[0], H.wb[0], single(C));
        else H.sap(0, H.wa[0], H.wb[0], 1, false, single(C));
    }
    HIPX(hipEventRecord(b, C->s));
    HIPX(hipGetLastError());
    HIPX(hipEventSynchronize(b));
    float ms = 0;
    HIPX(hipEventElapsedTime(&ms, a, b));
    C->ev_pool.push_back(a);
    C->ev_pool.push_back(b);
    return ms / reps;
}

// mean duration of the FP64 stencil applied to nr vectors at once (or of a
// plain FP64 copy of one vector, DD_K_BLAS) on random data
static double time_dirac64(dd_ctx* ctx, int cls, int nr, int reps) {
    const long n = 24L * ctx->g0.vh;
    Arena tmp;
    cx<double>* a = tmp.get<cx<double>>(n * nr);
    cx<double>* b = tmp.get<cx<double>>(n * nr);
    fine_random<double>(ctx->g0, nr, 12345ULL, 7, a, ctx->s);
    FineOp<double> op = fine_op<double>(ctx);
    auto launch = [&]() {
        if (cls == DD_K_BLAS) vec_convert<double, double>(n, a, b, ctx->s);
        else fine_dirac<double>(op, a, b, ctx->s, nr, n, all_rhs());
    };
    launch();
    hipEvent_t e0 = ev_get(ctx), e1 = ev_get(ctx);
    HIPX(hipEventRecord(e0, ctx->s));
    for (int r = 0; r < reps; r++) launch();
    HIPX(hipEventRecord(e1, ctx->s));
    HIPX(hipGetLastError());
    HIPX(hipEventSynchronize(e1));
    float ms = 0;
    HIPX(hipEventElapsedTime(&ms, e0, e1));
    ctx->ev_pool.push_back(e0);
    ctx->ev_pool.push_back(e1);
    return ms / reps;
}

dd_status dd_time_kernel(dd_ctx* ctx, int cls, int reps, double* avg_ms) {
    ABI_TRY(ctx)
    if (reps < 1 || !avg_ms) fail(DD_EINVAL, "reps >= 1 and avg_ms required");
    if (cls == DD_K_DIRAC64 || cls == DD_K_BLAS) {
        *avg_ms = time_dirac64(ctx, cls, 1, reps);
        return DD_OK;
    }
    if (cls == DD_K_COARSE) {
        // D_c on level 1 applied to max_rhs random vectors at once
        if (!ctx->have_setup) fail(DD_ESTATE, "the coarse stencil is timed after dd_setup");
        auto go = [&](auto& H) {
            const int k = ctx->R;
            coarse_random(H.g[1], H.nd[1], k, 4242ULL, 9, H.wa[1], ctx->s);
            const Batch bt{k, ctx->dflags + DI_ONES, (1u << k) - 1};
            H.apply_D(1, H.wa[1], H.wb[1], bt);
            hipEvent_t e0 = ev_get(ctx), e1 = ev_get(ctx);
            HIPX(hipEventRecord(e0, ctx->s));
            for (int r = 0; r < reps; r++) H.apply_D(1, H.wa[1], H.wb[1], bt);
            HIPX(hipEventRecord(e1, ctx->s));
            HIPX(hipGetLastError());
            HIPX(hipEventSynchronize(e1));
            float ms = 0;
            HIPX(hipEventElapsedTime(&ms, e0, e1));
            ctx->ev_pool.push_back(e0);
            ctx->ev_pool.push_back(e1);
            *avg_ms = ms / reps;
        };
        if (ctx->H64) go(*ctx->H64);
        else go(*ctx->H32);
        return DD_OK;
    }
    if (cls != DD_K_DIRAC_PREC && cls != DD_K_SAP) fail(DD_EINVAL, "kernel class not timed standalone");
    if (!ctx->configured) fail(DD_ESTATE, "dd_configure first");
    *avg_ms = ctx->H64 ? time_prec(ctx, *ctx->H64, cls, reps) : time_prec(ctx, *ctx->H32, cls, reps);
    return DD_OK;
    ABI_END(ctx)
}

long long dd_device_bytes(const dd_ctx* ctx) { return ctx ? ctx->fields.bytes + ctx->levels.bytes : 0; }

// op on k vectors (canonical [k][vol][nd] in and out) as one batch
template <class T>
static void apply_impl(dd_ctx* C, Hier<T>& H, int op, int l, int arg, int k, const double* in, double* out,
                       long* iters) {
    if (l < 0 || l >= H.nlev) fail(DD_EINVAL, "level out of range");
    if (k < 1 || k > C->R) fail(DD_EINVAL, "batch of " + std::to_string(k) + " vectors; max_rhs is " + std::to_string(C->R));
    long its[MAX_RHS] = {0};
    auto imp = [&](int lev, const double* src, cx<T>* dst) {
        if (lev == 0) fine_import_vectors<T>(H.g[0], k, src, dst, C->s);
        else coarse_import_vector<T>(H.g[lev], H.nd[lev], k, src, dst, C->s);
    };
    auto exp_ = [&](int lev, const cx<T>* src, double* dst) {
        if (lev == 0) fine_export_vectors<T>(H.g[0], k, src, dst, C->s);
        else coarse_export_vector<T>(H.g[lev], H.nd[lev], k, src, dst, C->s);
    };
    auto counts = [&](int lev) {
        for (int r = 0; r < k; r++) its[r] = H.coarse_count[lev][r];
    };
    const int bottom = H.nlev - 1;
    const Batch bt{k, C->dflags + DI_ONES, (1u << k) - 1};
    // precision 16: the fine-level V-cycle components run on FP16 spinor sets,
    // as in the solve (packed from and unpacked to the FP32 staging sets)
    const bool h16 = H.half && l == 0;
    auto pack = [&](const cx<T>* src, hspin dst) { fine_hpack<T>(H.g[0].vh, src, dst, H.nlv(0), k, bt.mask(), C->s); };
    auto unpack = [&](hspin src, cx<T>* dst) { fine_hunpack<T>(H.g[0].vh, src, dst, H.nlv(0), k, bt.mask(), C->s); };
    switch (op) {
        case DD_OP_D:
            if (l == 0) {
                const long n = 24L * C->g0.vh;
                cx<double>* a = C->ot;
                cx<double>* b = C->ot + (size_t)C->R * n;
                fine_import_vectors<double>(C->g0, k, in, a, C->s);
                fine_dirac<double>(fine_op<double>(C), a, b, C->s, k, n, bt.mask());
                fine_export_vectors<double>(C->g0, k, b, out, C->s);
                break;
            }
            imp(l, in, H.wa[l]);
            H.apply_D(l, H.wa[l], H.wb[l], bt);
            exp_(l, H.wb[l], out);
            break;
        case DD_OP_D_PREC:
            imp(0, in, H.wa[0]);
            H.apply_D(0, H.wa[0], H.wb[0], bt);
            exp_(0, H.wb[0], out);
            break;
        case DD_OP_SAP:
            if (l >= bottom) fail(DD_EINVAL, "no SAP on the coarsest level");
            imp(l, in, H.wa[l]);
            if (h16) {
                pack(H.wa[0], H.as_h(H.wb[0]));
                H.sap(0, H.as_h(H.wb[0]), H.as_h(H.wc[0]), arg, true, bt);
                unpack(H.as_h(H.wc[0]), H.wb[0]);
            } else {
                H.sap(l, H.wa[l], H.wb[l], arg, true, bt);
            }
            exp_(l, H.wb[l], out);
            break;
        case DD_OP_VCYCLE:
            if (l >= bottom) fail(DD_EINVAL, "no V-cycle on the coarsest level");
            if (!C->have_setup) fail(DD_ESTATE, "hierarchy not built");
            imp(l, in, H.wa[l]);
            memset(H.coarse_count, 0, sizeof H.coarse_count);
            if (h16) {
                pack(H.wa[0], H.as_h(H.wb[0]));
                H.vcycle(0, bottom, H.as_h(H.wb[0]), H.as_h(H.wc[0]), bt);
                unpack(H.as_h(H.wc[0]), H.wb[0]);
            } else {
                H.vcycle(l, bottom, H.wa[l], H.wb[l], bt);
            }
            counts(l + 1);
            exp_(l, H.wb[l], out);
            break;
        case DD_OP_RESTRICT:
            if (l >= bottom) fail(DD_EINVAL, "no restriction from the coarsest level");
            imp(l, in, H.wa[l]);
            if (h16) {
                pack(H.wa[0], H.as_h(H.wb[0]));
                H.restrict_(0, H.as_h(H.wb[0]), H.wa[1], bt);
            } else {
                H.restrict_(l, H.wa[l], H.wa[l + 1], bt);
            }
            exp_(l + 1, H.wa[l + 1], out);
            break;
        case DD_OP_PROLONG:
            if (l >= bottom) fail(DD_EINVAL, "no prolongation to the coarsest level");
            imp(l + 1, in, H.wa[l + 1]);
            if (h16) {
                H.prolong(0, H.wa[1], H.as_h(H.wc[0]), bt);
                unpack(H.as_h(H.wc[0]), H.wa[0]);
            } else {
                H.prolong(l, H.wa[l + 1], H.wa[l], bt);
            }
            exp_(l, H.wa[l], out);
            break;
        case DD_OP_COARSE_SOLVE:
            if (l < 1) fail(DD_EINVAL, "coarse solve needs level >= 1");
            imp(l, in, H.rc[l]);
            memset(H.coarse_count, 0, sizeof H.coarse_count);
            H.gmres_oe(l, H.rc[l], H.ec[l], bt);
            counts(l);
            exp_(l, H.ec[l], out);
            break;
        case DD_OP_SCHUR:
            if (l < 1) fail(DD_EINVAL, "Schur complement needs level >= 1");
            if (H.lexl[l]) fail(DD_EINVAL, "no odd-even Schur complement on a lattice with an odd extent");
            imp(l, in, H.wa[l]);
            H.schur(l, H.wa[l], H.wb[l], bt.mask(), k, k);
            for (int r = 0; r < k; r++)
                HIPX(hipMemsetAsync(H.wb[l] + (size_t)r * H.nlv(l), 0, sizeof(cx<T>) * (size_t)H.g[l].vh * H.nd[l], C->s));
            exp_(l, H.wb[l], out);
            break;
        case DD_OP_BICGSTAB: {
            if (l != 0 || k != 1) fail(DD_EINVAL, "odd-even BiCGStab acts on one fine vector (level 0)");
            if (arg < 1) fail(DD_EINVAL, "BiCGStab needs arg >= 1 steps");
            OeBicg<T> B = OeBicg<T>::make(C);
            imp(0, in, H.wa[0]);
            its[0] = B.apply(H.wa[0], H.wb[0], arg);
            exp_(0, H.wb[0], out);
            break;
        }
        case DD_OP_DEFLATED:
            if constexpr (std::is_same<T, double>::value) {
                if (l != 0 || k != 1) fail(DD_EINVAL, "the deflated operator acts on one fine vector (level 0)");
                if (H.nlev != 2 || !C->have_setup) fail(DD_ESTATE, "the deflated operator needs a built two-level setup");
                IdDefl Dp = IdDefl::make(C, &H, C->p.coarse_tol);
                memset(H.coarse_count, 0, sizeof H.coarse_count);
                fine_import_vectors<double>(C->g0, 1, in, Dp.b0, C->s);
                Dp.deflated(Dp.b0, Dp.chi1, bt);
                counts(1);
                fine_export_vectors<double>(C->g0, 1, Dp.chi1, out, C->s);
            } else {
                fail(DD_ESTATE, "the deflated operator runs on an FP64 setup");
            }
            break;
        case DD_OP_FGMRES:
            if (l < 1 || l >= bottom) fail(DD_EINVAL, "middle-level FGMRES needs 1 <= level < levels-1");
            imp(l, in, H.rc[l]);
            memset(H.coarse_count, 0, sizeof H.coarse_count);
            H.fgmres_mid(l, bottom, H.rc[l], H.ec[l], bt);
            counts(l);
            exp_(l, H.ec[l], out);
            break;
        default:
            fail(DD_EINVAL, "unknown op");
    }
    HIPX(hipGetLastError());
    sync(C);
    if (iters)
        for (int r = 0; r < k; r++) iters[r] = its[r];
}

dd_status dd_apply_batch(dd_ctx* ctx, int op, int level, int arg, int k, const double* in, double* out, long* iters) {
    ABI_TRY(ctx)
    if (!in || !out) fail(DD_EINVAL, "NULL vector");
    if (!ctx->configured) fail(DD_ESTATE, "dd_configure first");
    if (ctx->H64) apply_impl(ctx, *ctx->H64, op, level, arg, k, in, out, iters);
    else apply_impl(ctx, *ctx->H32, op, level, arg, k, in, out, iters);
    return DD_OK;
    ABI_END(ctx)
}

dd_status dd_apply(dd_ctx* ctx, int op, int level, int arg, const double* in, double* out, long* iters) {
    ABI_TRY(ctx)
    if (!in || !out) fail(DD_EINVAL, "NULL vector");
    if (!ctx->configured) {
        if (op == DD_OP_D && level == 0) {
            const long n = 24L * ctx->g0.vh;
            Arena tmp;
            cx<double>* a = tmp.get<cx<double>>(n);
            cx<double>* b = tmp.get<cx<double>>(n);
            fine_import_spinor<double>(ctx->g0, in, a, ctx->s);
            fine_dirac<double>(fine_op<double>(ctx), a, b, ctx->s);
            fine_export_spinor<double>(ctx->g0, b, out, ctx->s);
            HIPX(hipGetLastError());
            sync(ctx);
            return DD_OK;
        }
        fail(DD_ESTATE, "dd_configure first");
    }
    if (ctx->H64) apply_impl(ctx, *ctx->H64, op, level, arg, 1, in, out, iters);
    else apply_impl(ctx, *ctx->H32, op, level, arg, 1, in, out, iters);
    return DD_OK;
    ABI_END(ctx)
}



dd_status dd_apply_D_noalloc(dd_ctx* ctx, const double* in, double* out) {
    ABI_TRY(ctx)
    if (!in || !out) fail(DD_EINVAL, "NULL vector");
    if ((size_t)ctx->vol > NOALLOC_SITES)
        fail(DD_EINVAL, "lattice of " + std::to_string(ctx->vol) + " sites exceeds the allocation-free limit of " +
                            std::to_string(NOALLOC_SITES) + " sites");
    if (!ctx->scratch) fail(DD_EDEVICE, "scratch array unavailable: " + ctx->scratch_err);
    const long n = 24L * ctx->g0.vh;   // complex entries of one fine spinor
    cx<double>* a = reinterpret_cast<cx<double>*>(ctx->scratch);
    cx<double>* b = a + n;
    // the import writes every entry of a and the stencil every entry of b:
    // nothing has to start at zero
    fine_import_spinor<double>(ctx->g0, in, a, ctx->s);
    fine_dirac<double>(fine_op<double>(ctx), a, b, ctx->s);
    fine_export_spinor<double>(ctx->g0, b, out, ctx->s);
    HIPX(hipGetLastError());
    HIPX(hipStreamSynchronize(ctx->s));
    return DD_OK;
    ABI_END(ctx)
}

static void set_sched(dd_ctx* C, int sched) {
    C->sched = sched;
    // captured graphs hold the previous kernel choices
    auto drop = [](auto& H) {
        for (auto& kv : H.graphs) (void)hipGraphExecDestroy(kv.second);
        H.graphs.clear();
    };
    if (C->H64) drop(*C->H64);
    if (C->H32) drop(*C->H32);
    // a new schedule tries the cooperative cycle again
    if (C->H64) C->H64->coop_off = false;
    if (C->H32) C->H32->coop_off = false;
    const int mf = (sched & SCHED_NO_MFMA) ? 0 : 1;
    if (C->H64) {
        C->H64->op0.sched = sched;
        for (int l = 0; l < DD_MAXLEV; l++) C->H64->cop[l].mfma = mf;
    }
    if (C->H32) {
        C->H32->op0.sched = C->H32->op0h.sched = sched;
        for (int l = 0; l < DD_MAXLEV; l++) C->H32->cop[l].mfma = C->H32->coph[l].mfma = mf;
    }
}

dd_status dd_set_schedule(dd_ctx* ctx, int sched) {
    ABI_TRY(ctx)
    if (sched < 0 || sched > (SCHED_FUSED | SCHED_XCD | SCHED_LDS | SCHED_NO_MFMA | SCHED_GRAPH | SCHED_COOP |
                              SCHED_COOP_ABORT))
        fail(DD_EINVAL, "unknown schedule flags");
    set_sched(ctx, sched);
    return DD_OK;
    ABI_END(ctx)
}

int dd_get_schedule(const dd_ctx* ctx) { return ctx ? ctx->sched : -1; }

// Autotuner: every schedule is timed on the context's own fields (FP64
// stencil, plus nu SAP sweeps in preconditioner precision once configured,
// the fine-level work of one outer iteration); the fastest one is kept.
dd_status dd_autotune(dd_ctx* ctx, int reps, int* chosen, double* times_ms) {
    ABI_TRY(ctx)
    if (reps < 1) fail(DD_EINVAL, "reps >= 1");
    const int nsched = (SCHED_FUSED | SCHED_XCD | SCHED_LDS) + 1;
    const int keep = ctx->sched & (SCHED_NO_MFMA | SCHED_GRAPH | SCHED_COOP);
    double best = 0;
    int pick = ctx->sched;
    // the outer stencil is timed at the batch width of the solves, up to four
    // (the XCD-ordered schedules let the workgroups of one block's RHS share
    // L2; four show it, and the two temporary vector sets stay small)
    const int nr = ctx->configured ? std::min(std::max(ctx->R, 1), 4) : 1;
    for (int sc = 0; sc < nsched; sc++) {
        set_sched(ctx, sc | keep);
        double ms = time_dirac64(ctx, DD_K_DIRAC64, nr, reps) / nr, t = 0;
        if (ctx->configured) {
            if (dd_time_kernel(ctx, DD_K_SAP, reps, &t) != DD_OK) return DD_EDEVICE;
            ms += std::max(ctx->p.nu, 1) * t;
        }
        if (times_ms) times_ms[sc] = ms;
        if (sc == 0 || ms < best) { best = ms; pick = sc | keep; }
    }
    set_sched(ctx, pick);
    if (chosen) *chosen = pick;
    return DD_OK;
    ABI_END(ctx)
}

// Coarse-solver autotuner: one coarsest-level solve on a fixed random RHS with
// step-by-step launches (single kernel launches, then chunks of steps replayed
// as graphs) and with the cooperative cycle at 16, 32, 64 and 128 workgroups;
// the fastest is kept.
template <class T>
static void tune_coarse(dd_ctx* C, Hier<T>& H, int reps, int* chosen, double* times) {
    const int l = H.nlev - 1;
    coarse_random(H.g[l], H.nd[l], 1, 777ULL, 11, H.rc[l], C->s);
    const Batch one = single(C);
    constexpr int NV = 6;
    const int caps[NV] = {0, 0, 16, 32, 64, 128};
    const int saved = C->sched & ~(SCHED_COOP | SCHED_GRAPH), saved_cap = C->coop_cap;
    auto flags = [&](int v) {
        return v == 0 ? saved : v == 1 ? (saved | SCHED_GRAPH) : (saved | SCHED_GRAPH | SCHED_COOP);
    };
    double best = 0;
    int pick = 0;
    for (int v = 0; v < NV; v++) {
        C->sched = flags(v);
        C->coop_cap = caps[v] ? caps[v] : saved_cap;
        H.coop_off = false;
        H.gmres_oe(l, H.rc[l], H.ec[l], one);   // warm-up (graph capture)
        sync(C);
        const double t0 = now_s();
        for (int r = 0; r < reps; r++) H.gmres_oe(l, H.rc[l], H.ec[l], one);
        sync(C);
        const double ms = (now_s() - t0) * 1e3 / reps;
        if (times) times[v] = ms;
        if (v == 0 || ms < best) { best = ms; pick = v; }
    }
    // single launches and graph replay compare in context, by whole outer
    // solves of a random right-hand side: the graph's launch latency and how
    // far the host's enqueueing runs ahead both depend on the work around the
    // coarse solves
    if (times) times[NV] = times[NV + 1] = 0.0;
    if (caps[pick] == 0) {
        fine_random<double>(C->g0, 1, 778ULL, 12, C->ob, C->s);
        double ts[2];
        for (int v = 0; v < 2; v++) {
            C->sched = flags(v);
            C->coop_cap = saved_cap;
            dd_stats sb[MAX_RHS];
            dd_status rc[MAX_RHS];
            outer_fgmres<T>(C, H, 1, 1e-10, 0, sb, rc);   // warm-up (graph capture)
            sync(C);
            const double t0 = now_s();
            for (int r = 0; r < reps; r++) outer_fgmres<T>(C, H, 1, 1e-10, 0, sb, rc);
            sync(C);
            ts[v] = (now_s() - t0) * 1e3 / reps;
            if (times) times[NV + v] = ts[v];
        }
        pick = (ts[1] < ts[0]) ? 1 : 0;
    }
    C->sched = flags(pick);
    C->coop_cap = caps[pick] ? caps[pick] : saved_cap;
    memset(H.coarse_count, 0, sizeof H.coarse_count);
    if (chosen) *chosen = caps[pick];
}

dd_status dd_autotune_coarse(dd_ctx* ctx, int reps, int* chosen_grid, double* times_ms) {
    ABI_TRY(ctx)
    if (reps < 1) fail(DD_EINVAL, "reps >= 1");
    if (!ctx->have_setup) fail(DD_ESTATE, "the coarse solver is tuned after dd_setup");
    if (ctx->H64) tune_coarse(ctx, *ctx->H64, reps, chosen_grid, times_ms);
    else tune_coarse(ctx, *ctx->H32, reps, chosen_grid, times_ms);
    return DD_OK;
    ABI_END(ctx)
}


// ---------------------------------------------------------------------------
// Persistent autotuning cache: one text line per tuned problem shape,
//   <key> TAB <schedule flags> <cooperative workgroups>
// The key names the device (architecture, compute units) and everything the
// launch forms' costs depend on: lattice, precision, max_rhs, levels, test
// vectors, aggregates and SAP blocks per level, MR steps and nu.  The choices
// are launch forms whose results agree to rounding, so a stored choice serves
// every field and mass of the same shape.
// ---------------------------------------------------------------------------
static std::string tune_key(dd_ctx* C) {
    int dev = 0;
    HIPX(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPX(hipGetDeviceProperties(&prop, dev));
    const dd_params& p = C->p;
    std::string k = std::string(prop.gcnArchName) + ":" + std::to_string(prop.multiProcessorCount) + "cu";
    k += " dims=" + std::to_string(C->dims[0]) + "x" + std::to_string(C->dims[1]) + "x" + std::to_string(C->dims[2]) +
         "x" + std::to_string(C->dims[3]);
    k += " prec=" + std::to_string(p.precision) + " rhs=" + std::to_string(p.max_rhs) + " lev=" +
         std::to_string(p.levels) + " nu=" + std::to_string(p.nu);
    for (int l = 0; l + 1 < p.levels; l++) {
        k += " L" + std::to_string(l) + "=n" + std::to_string(p.n_tv[l]) + ",a" + std::to_string(p.agg[l][0]);
        for (int mu = 1; mu < 4; mu++) k += "x" + std::to_string(p.agg[l][mu]);
        k += ",s" + std::to_string(p.sap[l][0]);
        for (int mu = 1; mu < 4; mu++) k += "x" + std::to_string(p.sap[l][mu]);
        k += ",mr" + std::to_string(p.mr_steps[l]);
    }
    return k;
}

dd_status dd_autotune_cached(dd_ctx* ctx, const char* path, int reps, int* sched, int* grid, int* hit) {
    ABI_TRY(ctx)
    if (!path || !*path) fail(DD_EINVAL, "NULL cache path");
    if (reps < 1) fail(DD_EINVAL, "reps >= 1");
    if (!ctx->have_setup) fail(DD_ESTATE, "the launch forms are tuned after dd_setup");
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    const std::string key = tune_key(ctx);
    int fs = -1, fg = -1;
    if (FILE* f = fopen(path, "r")) {
        char line[1024];
        while (fgets(line, sizeof line, f)) {
            char* tab = strchr(line, '\t');
            if (!tab) continue;
            *tab = 0;
            int a = -1, b = -1;
            if (key == line && sscanf(tab + 1, "%d %d", &a, &b) == 2 && a >= 0 && b >= 0) { fs = a; fg = b; }
        }
        fclose(f);
    }
    const bool found = fs >= 0;
    if (found) {
        set_sched(ctx, fs);
        if (fg > 0) ctx->coop_cap = fg;
    } else {
        dd_status rc = dd_autotune(ctx, reps, nullptr, nullptr);
        if (rc != DD_OK) return rc;
        rc = dd_autotune_coarse(ctx, reps, &fg, nullptr);
        if (rc != DD_OK) return rc;
        fs = ctx->sched;
        FILE* f = fopen(path, "a");
        if (!f) fail(DD_EINVAL, std::string("cannot append to the autotuning cache ") + path + " (the tuned forms are in use)");
        fprintf(f, "%s\t%d %d\n", key.c_str(), fs, fg);
        fclose(f);
    }
    if (sched) *sched = ctx->sched;
    if (grid) *grid = fg;
    if (hit) *hit = found ? 1 : 0;
    return DD_OK;
    ABI_END(ctx)
}
