// Host engine and C ABI of the HOTRG library (include/hotrg.h).
//
// One context = one coarse-graining state in device memory.  A step along mu
// (Sec. 2; Eqs. (2.8)-(2.9) in four dimensions) runs entirely on the device:
//   1. squeezed environments of the merged transverse legs from two Grams each
//      (HOSVD of the merged tensor), FP64;
//   2. Jacobi eigendecomposition of every environment, FP64;
//   3. (host, on the spectra only) truncation and side choice;
//   4. for every K slice (alpha, a1'): isometry products build the operand
//      rows A_s (T, S_m, S_e stacked) and columns B_s, then the MFMA GEMM
//      accumulates C += A_s B_s^T;
//   5. Frobenius norm c_n of the T block, then C is permuted back to the
//      canonical leg order and divided by c_n.
// Index names follow the paper: for a step along mu the transverse axes are
// a, b, c (increasing axis id); T1 legs (a1, a1', b1, b1', c1, c1', mu1,
// alpha), T2 legs (a2, a2', b2, b2', c2, c2', alpha, mu2'); new legs a = U
// over (a1, a2), a' = U over (a1', a2'), etc.
#include "../../include/hotrg.h"
#include "hotrg_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

using namespace hotrg;

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

struct Decision {
    int side = -1;
    int k = 0;
    double eps_b = 0, eps_f = 0, gap = INFINITY;
    bool flagged = false;
    bool truncated = false;
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

constexpr double kSideTie = 1e-11;
// an eigensolve that reaches the sweep cap still counts as converged when the
// squared off-diagonal norm it leaves is below this fraction of the total
constexpr double kEigResidOk = 1e-24;
constexpr int kMaxEnvN = 169;  // environments of D^2 x D^2, D <= 13

}  // namespace

struct hotrg_ctx {
    double beta = 0, h = 0;
    int dcut = 0;
    hotrg_config cfg{};
    hipStream_t stream = nullptr;
    bool failed = false;

    int dims[4] = {2, 2, 2, 2};
    int n = 0;
    int first_axis = -1, last_axis = -1;
    double lnz_acc = 0;
    size_t cap = 0;  // elements of the largest tensor, max(2, dcut)^8

    double *state[3] = {nullptr, nullptr, nullptr};  // T, S_m, S_e (canonical layout)
    double *cbuf = nullptr;                          // 3 * cap: GEMM output rows T | S_m | S_e
    double *gram_x = nullptr;                        // cap
    double *y1 = nullptr, *y2 = nullptr;             // cap each
    double *gram_part = nullptr;
    size_t gram_part_cap = 0;
    double *G = nullptr;     // 2 * 169^2 (one pair of Grams at a time)
    double *E = nullptr;     // 6 * 169^2
    double *lam = nullptr;   // 6 * 169
    double *V = nullptr;     // 6 * 169^2
    double *jwork = nullptr; // 2 * 2 * 145^2
    int *sweeps = nullptr;
    double *resid = nullptr;
    double *U[3] = {nullptr, nullptr, nullptr};  // chosen isometries, 169^2 each, row-major n x k
    double *partials = nullptr;                   // 1024
    double *scal = nullptr;                       // 64
    double *obs = nullptr;                        // 3 + 169
    DevBuf f64_slices;                            // FP64 operand slices
    DevBuf x3_slices;                             // bf16 hi/lo operand slices
    DevBuf gemm_tail;                             // second k-halves of the GEMM's last round of tiles
    std::vector<DevBuf> owned;

    // host-side record of the last step
    Decision dec[4];
    std::vector<double> spectra[4][2];
    int Urows[4] = {0, 0, 0, 0}, Ucols[4] = {0, 0, 0, 0};
    double min_gap = INFINITY;
    int flagged = 0;
    double last_cn = 0;
    int iso_axis = -1;       // axis of the step the current isometries belong to
    int eig_sweeps = 0;      // most Jacobi sweeps of one solve in the last step
    double eig_resid = 0;    // largest off-diagonal / total squared norm left by those solves

    // GEMM timing
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double gemm_ms = 0;
    long long gemm_launches = 0;
    long long z2_tile_launches = 0;  // last isometry products run in the tile form of the Z2 scatter
    long long z2_rev_steps = 0;      // reverse-pass steps undone in the Z2 block form
    // tile form of the Z2 scatter, per last product (0: A rows, 1: B rows of
    // the forward; 2, 3: the transposed A, B operands of the reverse pass):
    // the slot table and the compacted isometry block, rebuilt once per set of
    // class tables (z2_gen counts the table builds)
    long long z2_gen = 0, tile_gen[4] = {-1, -1, -1, -1};
    std::vector<uint32_t> tperm_h[4];
    std::vector<int32_t> tidx_h[4];  // compacted isometry block: source offsets (-1: zero)
    uint32_t *tperm_d[4] = {};
    int32_t *tidx_d[4] = {};
    double *tU_d[4] = {};
    uint32_t tslots[4] = {};
    int tNH[4] = {};
    uint32_t tlab1[4] = {}, tlab2[4] = {}, tnI[4][2] = {};
    uint64_t tI[4][2] = {};
    // reverse pass, block form: the inner K indices of the transposed B
    // operand in the order (b1', a2, b2, c2, c1') (host / device), and its
    // entries listed in the dense order (the A_bar table)
    std::vector<uint32_t> ktabq_h, kmapq_h;
    uint32_t *ktabq = nullptr, *kmapq = nullptr;
    double gemm_flops = 0;
    size_t device_bytes = 0;
    // phase timing of hotrg_step: events at the start, after the isometries,
    // after the contraction and after the normalisation (device timeline)
    hipEvent_t ph[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ph_pending = false;
    double phase_ms[3] = {0, 0, 0};
    long long phase_steps = 0;

    // Z2 parity of every bond index (h = 0): valid while z2 is set.  A step
    // whose isometry columns each lie in one parity sector keeps it (the new
    // labels are those sectors); the contraction of such a step runs in the
    // block form (step_z2) unless dense_only is configured.
    bool z2 = false;
    std::vector<uint8_t> par[4];
    std::vector<uint8_t> new_par[4];
    bool step_z2 = false;
    struct Z2Layout {
        uint32_t N[2];      // rows (= columns) of one tensor per parity class
        uint32_t Kc[2];     // inner K indices per parity class
        uint64_t ldk[2];    // operand row length per class (bf16: padded to 64)
        uint32_t R[2];      // stacked A rows of GEMM class g
        uint64_t coff[2];   // offset of C_g in cbuf
    } z2l{};
    std::vector<uint32_t> rtab_h, ktab_h;  // host copies (kept alive for the uploads)
    uint32_t *rtab = nullptr, *ktab = nullptr;
    DevBuf z2_slices;

    // per-step checkpoints for the reverse pass (keep_checkpoints = 1)
    struct Checkpoint {
        int dims[4];
        int axis;
        int tv[3];
        int k[3];
        int n[3];         // n = D^2 of each transverse axis
        int side[3];      // environment side the isometry came from
        bool trunc[3];    // isometry from an eigendecomposition (else constant)
        bool flagged[3];  // the cut stayed inside a degenerate multiplet (no gap above tau)
        double c;         // c_n of the step
        bool z2 = false;  // the step contracted in the Z2 block form (its labels below)
        std::vector<uint8_t> par[4];   // parity labels of the bonds before the step
        std::vector<uint8_t> npar[3];  // labels of the new transverse bonds (axis tv[i])
        double *T;        // state before the step
        double *U[3];     // n x k
        double *lam[3];   // n (chosen side, descending)
        double *V[3];     // n x n
    };
    std::vector<Checkpoint> ckpts;
    Checkpoint pending{};
    bool ckpt_broken = false;
    double c0 = 1.0;
    // reverse-pass work buffers
    DevBuf bw[18];
    uint32_t *rev_tabs = nullptr;  // reverse pass, block form: class lists and Tbar offsets of the rows
    double *xmv_buf = nullptr;     // reverse pass: the gathered small matrix of a small-matrix product
};

namespace {

#define HIP_TRY(ctx, call)                                                                          \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            (ctx)->failed = true;                                                                   \
            return set_err(HOTRG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));       \
        }                                                                                           \
    } while (0)

#define TRY(expr)                  \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != HOTRG_OK) return rc_; \
    } while (0)

// Every device buffer of a context comes from here: the caller's allocator
// (hotrg_config.alloc / free, e.g. a framework's caching allocator) when one
// is given, else hipMalloc.  mem_budget caps the bytes held at once.
int dev_alloc(hotrg_ctx *c, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) / 256 * 256;
    if (c->cfg.mem_budget > 0 && c->device_bytes + bytes > c->cfg.mem_budget)
        return set_err(HOTRG_ENOMEM, "allocation of " + std::to_string(bytes) + " bytes would exceed mem_budget (" +
                                         std::to_string(c->cfg.mem_budget) + " bytes, " +
                                         std::to_string(c->device_bytes) + " held)");
    if (c->cfg.alloc) {
        *p = c->cfg.alloc(bytes, c->cfg.alloc_ctx);
        if (!*p) return set_err(HOTRG_ENOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return set_err(HOTRG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                             hipGetErrorString(e));
        }
    }
    c->owned.push_back(DevBuf{*p, bytes});
    c->device_bytes += bytes;
    return HOTRG_OK;
}

void release(hotrg_ctx *c, void *p) {
    if (c->cfg.free) c->cfg.free(p, c->cfg.alloc_ctx);
    else (void)hipFree(p);
}

// Returns one buffer obtained from dev_alloc (the stream must be idle with
// respect to it).  Unknown or null pointers are ignored.
void dev_free(hotrg_ctx *c, void *p) {
    if (!p) return;
    for (size_t i = 0; i < c->owned.size(); ++i)
        if (c->owned[i].p == p) {
            c->device_bytes -= c->owned[i].bytes;
            release(c, p);
            c->owned[i] = c->owned.back();
            c->owned.pop_back();
            return;
        }
}

template <typename T>
int alloc_n(hotrg_ctx *c, T **p, size_t count) {
    return dev_alloc(c, (void **)p, count * sizeof(T));
}

int ensure(hotrg_ctx *c, DevBuf &b, size_t bytes) {
    if (b.bytes >= bytes) return HOTRG_OK;
    if (b.p) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dev_free(c, b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    void *p = nullptr;
    TRY(dev_alloc(c, &p, bytes));
    b.p = p;
    b.bytes = bytes;
    return HOTRG_OK;
}

PermParams perm_params(int nd, const int *ext, const uint32_t *in_st, uint64_t *max_in = nullptr) {
    PermParams p{};
    p.nd = nd;
    uint64_t total = 1, mx = 0;
    for (int k = 0; k < nd; ++k) {
        p.ext[k] = make_fastdiv((uint32_t)ext[k]);
        p.in_st[k] = in_st[k];
        total *= (uint64_t)ext[k];
        mx += (uint64_t)(ext[k] - 1) * in_st[k];
    }
    p.total = (uint32_t)total;
    if (max_in) *max_in = mx;
    return p;
}

// Isometry expand-product description (see ExpandParams).
struct XP {
    ExpandParams p{};
    uint64_t threads = 1, max_in = 0, max_u = 0, max_out = 0;
    bool bad = false;
    void tdim(int ext, uint64_t ist, uint64_t ost) {
        if (p.nd >= XP_MAXD) {
            bad = true;
            return;
        }
        int k = p.nd++;
        p.ext[k] = make_fastdiv((uint32_t)ext);
        p.in_st[k] = (uint32_t)ist;
        p.out_st[k] = (uint32_t)ost;
        threads *= (uint64_t)ext;
        max_in += (uint64_t)(ext - 1) * ist;
        max_out += (uint64_t)(ext - 1) * ost;
    }
    void loops(int L1, uint64_t u1, uint64_t o1, int L2, uint64_t u2, uint64_t o2) {
        p.L1 = L1;
        p.L2 = L2;
        p.u1 = (uint32_t)u1;
        p.o1 = (uint32_t)o1;
        p.u2 = (uint32_t)u2;
        p.o2 = (uint32_t)o2;
        max_u += (uint64_t)(L1 - 1) * u1 + (uint64_t)(L2 - 1) * u2;
        max_out += (uint64_t)(L1 - 1) * o1 + (uint64_t)(L2 - 1) * o2;
    }
    void sum(int n, uint64_t xs, uint64_t us) {
        p.nsum = n;
        p.xs = (uint32_t)xs;
        p.us = (uint32_t)us;
        max_in += (uint64_t)(n - 1) * xs;
        max_u += (uint64_t)(n - 1) * us;
    }
    // host-side bounds check (elements available from each base pointer)
    bool fits(uint64_t in_avail, uint64_t u_avail, uint64_t out_avail) const {
        return !bad && p.nsum >= 1 && p.nsum <= XP_MAXS && p.L1 >= 1 && p.L2 >= 1 && p.L2 <= XP_MAXS &&
               threads < (1ull << 31) && max_in < in_avail && max_in < (1ull << 32) && max_u < u_avail &&
               max_out < out_avail && max_out < (1ull << 32);
    }
    // bf16 outputs go to the packed GEMM layout of a row-major operand with row length ld
    void packed(uint64_t ld, uint32_t row0 = 0) {
        p.pack = 1;
        p.pld = make_fastdiv((uint32_t)ld);
        p.pkb = (uint32_t)(ld / PACK_K);
        p.prow0 = row0;
    }
    const ExpandParams &done() {
        p.threads = (uint32_t)threads;
        return p;
    }
};

// Generic contraction description (see EinsumParams), with host bounds checks.
struct EP {
    EinsumParams p{};
    uint64_t nout = 1, S = 1, mx = 0, my = 0, mz = 0;
    bool bad = false;
    void o(int ext, uint64_t sx, uint64_t sy, uint64_t sz) {
        if (p.ndo >= EIN_MAXO) {
            bad = true;
            return;
        }
        int k = p.ndo++;
        p.oext[k] = make_fastdiv((uint32_t)ext);
        p.ox[k] = (uint32_t)sx;
        p.oy[k] = (uint32_t)sy;
        p.oz[k] = (uint32_t)sz;
        nout *= (uint64_t)ext;
        mx += (uint64_t)(ext - 1) * sx;
        my += (uint64_t)(ext - 1) * sy;
        mz += (uint64_t)(ext - 1) * sz;
    }
    void s(int ext, uint64_t sx, uint64_t sy) {
        if (p.nds >= EIN_MAXS) {
            bad = true;
            return;
        }
        int k = p.nds++;
        p.sext[k] = (uint32_t)ext;
        p.sx[k] = (uint32_t)sx;
        p.sy[k] = (uint32_t)sy;
        S *= (uint64_t)ext;
        mx += (uint64_t)(ext - 1) * sx;
        my += (uint64_t)(ext - 1) * sy;
    }
    bool fits(uint64_t xa, uint64_t ya, uint64_t za) const {
        return !bad && nout < (1ull << 31) && S < (1ull << 31) && mx < xa && my < ya && mz < za &&
               mx < (1ull << 32) && my < (1ull << 32) && mz < (1ull << 32);
    }
    EinsumParams done(double alpha, int accumulate) {
        p.nout = (uint32_t)nout;
        p.S = (uint32_t)S;
        p.alpha = alpha;
        p.accumulate = accumulate;
        return p;
    }
};

void row_major_strides(int nd, const int *ext, uint64_t *st) {
    uint64_t s = 1;
    for (int k = nd - 1; k >= 0; --k) {
        st[k] = s;
        s *= (uint64_t)ext[k];
    }
}

size_t tensor_size(const int D[4]) {
    size_t s = 1;
    for (int q = 0; q < 4; ++q) s *= (size_t)D[q] * D[q];
    return s;
}

// canonical element strides of the 8 legs for dims D
void canon_strides(const int D[4], uint64_t st[8]) {
    uint64_t s = 1;
    for (int l = 7; l >= 0; --l) {
        st[l] = s;
        s *= (uint64_t)D[l / 2];
    }
}

// Optional progress report for long steps (environment HOTRG_PROGRESS=1):
// about ten lines per contraction or reverse step, each printed after the
// stream has finished the slices it counts.
bool progress_enabled() {
    static const bool on = [] {
        const char *v = std::getenv("HOTRG_PROGRESS");
        return v && v[0] == '1';
    }();
    return on;
}

int report_progress(hotrg_ctx *c, const char *what, int step, int done, int total) {
    if (!progress_enabled() || total < 10) return HOTRG_OK;
    const int every = total / 10;
    if (done % every != 0 && done != total) return HOTRG_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::fprintf(stderr, "hotrg: step %d %s: %d / %d slices done\n", step, what, done, total);
    std::fflush(stderr);
    return HOTRG_OK;
}

hipEvent_t next_event(hotrg_ctx *c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Reading R3: cut at dcut unless the gap there is <= tau * lam_1; then the
// largest smaller k with a gap above tau.
Decision choose_cut(const double *lam, int n, int dcut, double tau) {
    Decision d;
    d.truncated = true;
    double l1 = lam[0];
    if (!(l1 > 0)) {
        d.k = dcut;
        d.gap = 0;
        d.flagged = true;
        return d;
    }
    auto gap = [&](int k) { return (lam[k - 1] - lam[k]) / l1; };
    if (gap(dcut) > tau) {
        d.k = dcut;
        d.gap = gap(dcut);
        return d;
    }
    for (int k = dcut - 1; k >= 1; --k)
        if (gap(k) > tau) {
            d.k = k;
            d.gap = gap(k);
            return d;
        }
    d.k = dcut;
    d.gap = gap(dcut);
    d.flagged = true;
    return d;
}

double discarded(const double *lam, int n, int k) {
    double e = 0;
    for (int i = k; i < n; ++i) e += std::max(lam[i], 0.0);
    return e;
}

// Gram of T with open legs (leg_p, leg_a) in local numbering; local leg l
// has canonical stride lst[l] and dimension ldim[l].  Result R x R with
// R = ldim[leg_p] * ldim[leg_a], row index p * Da + a.
int gram(hotrg_ctx *c, const double *T, const uint64_t lst[8], const int ldim[8], int leg_p, int leg_a, double *G) {
    int ext[8];
    uint32_t st[8];
    int nd = 0;
    ext[nd] = ldim[leg_p];
    st[nd++] = (uint32_t)lst[leg_p];
    ext[nd] = ldim[leg_a];
    st[nd++] = (uint32_t)lst[leg_a];
    size_t K = 1;
    for (int l = 0; l < 8; ++l) {
        if (l == leg_p || l == leg_a) continue;
        ext[nd] = ldim[l];
        st[nd++] = (uint32_t)lst[l];
        K *= (size_t)ldim[l];
    }
    int R = ldim[leg_p] * ldim[leg_a];
    uint64_t mx = 0;
    PermParams pp = perm_params(8, ext, st, &mx);
    if (mx >= c->cap || pp.total > c->cap || R > kMaxEnvN) return set_err(HOTRG_EINVAL, "gram launch out of bounds");
    launch_permute(pp, T, c->gram_x, 1.0, c->stream);
    int nchunks = (int)std::min<size_t>(std::max<size_t>(1, K / 512), 1024);
    size_t need = (size_t)nchunks * R * R;
    if (need > c->gram_part_cap) return set_err(HOTRG_ENOMEM, "gram partial buffer too small");
    launch_gram(c->gram_x, R, K, c->gram_part, nchunks, G, c->stream);
    return HOTRG_OK;
}

int check_launch(hotrg_ctx *c, const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->failed = true;
        return set_err(HOTRG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
    return HOTRG_OK;
}

// Environment + eigh + decisions for every transverse axis; fills c->U[i],
// k[i] (kept), and the decision record.  Local legs: 0..5 transverse
// (a, a', b, b', c, c'), 6 = mu1 (backward), 7 = mu' (forward).
int isometries(hotrg_ctx *c, const double *T, const uint64_t lst[8], const int ldim[8], const int tv[3], int mu,
               int k_out[3]) {
    const int Dm = ldim[6];
    for (int q = 0; q < 4; ++q) {
        c->dec[q] = Decision();
        c->spectra[q][0].clear();
        c->spectra[q][1].clear();
    }
    c->min_gap = INFINITY;
    c->flagged = 0;
    c->eig_sweeps = 0;
    c->eig_resid = 0;
    c->iso_axis = mu;
    for (int i = 0; i < 3; ++i) {
        const int D = ldim[2 * i];
        const int nmat = D * D;
        int q = tv[i];
        if (nmat <= c->dcut) {
            launch_identity(c->U[i], nmat, c->stream);
            k_out[i] = nmat;
            c->dec[q].k = nmat;
            c->Urows[q] = nmat;
            c->Ucols[q] = nmat;
            continue;
        }
        if (nmat > kMaxEnvN) return set_err(HOTRG_EINVAL, "environment larger than 169 x 169");
        double *Eb = c->E + (size_t)(2 * i) * kMaxEnvN * kMaxEnvN;
        for (int side = 0; side < 2; ++side) {
            int leg = 2 * i + side;
            double *G1 = c->G, *G2 = c->G + (size_t)kMaxEnvN * kMaxEnvN;
            TRY(gram(c, T, lst, ldim, leg, 7, G1));
            TRY(gram(c, T, lst, ldim, leg, 6, G2));
            launch_env_combine(G1, G2, D, D, Dm, Eb + (size_t)side * nmat * nmat, c->stream);
        }
        // both sides share n, so they go in one launch; matrices packed at stride n*n
        launch_jacobi_eigh(Eb, nmat, 2, c->lam + (size_t)2 * i * kMaxEnvN, c->V + (size_t)2 * i * kMaxEnvN * kMaxEnvN,
                           c->jwork, c->sweeps, c->resid, c->cfg.eig_max_sweeps, c->stream);
        TRY(check_launch(c, "environment / eigh"));
        std::vector<double> lam(2 * (size_t)nmat);
        int sw[2] = {0, 0};
        double rs[2] = {0, 0};
        HIP_TRY(c, hipMemcpyAsync(lam.data(), c->lam + (size_t)2 * i * kMaxEnvN, sizeof(double) * 2 * nmat,
                                  hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(sw, c->sweeps, sizeof(sw), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(rs, c->resid, sizeof(rs), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int side = 0; side < 2; ++side) {
            c->eig_sweeps = std::max(c->eig_sweeps, sw[side]);
            c->eig_resid = std::max(c->eig_resid, rs[side]);
            // the sweep cap was reached with an off-diagonal part above the
            // rounding level: the eigenvectors are not converged
            if (sw[side] >= c->cfg.eig_max_sweeps && !(rs[side] <= kEigResidOk)) {
                c->failed = true;
                return set_err(HOTRG_ENUMERIC,
                               "eigensolver did not converge in " + std::to_string(c->cfg.eig_max_sweeps) +
                                   " sweeps (environment of axis " + std::to_string(q) + ", side " +
                                   std::to_string(side) + ", n = " + std::to_string(nmat) +
                                   ", off-diagonal / total squared norm " + std::to_string(rs[side]) + ")");
            }
        }
        Decision db = choose_cut(lam.data(), nmat, c->dcut, c->cfg.tau_deg);
        Decision df = choose_cut(lam.data() + nmat, nmat, c->dcut, c->cfg.tau_deg);
        double eb = discarded(lam.data(), nmat, db.k), ef = discarded(lam.data() + nmat, nmat, df.k);
        double scale = discarded(lam.data(), nmat, 0);
        int side = (eb <= ef + kSideTie * scale) ? 0 : 1;
        Decision d = side == 0 ? db : df;
        d.side = side;
        d.eps_b = eb;
        d.eps_f = ef;
        c->dec[q] = d;
        c->spectra[q][0].assign(lam.begin(), lam.begin() + nmat);
        c->spectra[q][1].assign(lam.begin() + nmat, lam.end());
        c->min_gap = std::min(c->min_gap, d.gap);
        c->flagged |= d.flagged ? 1 : 0;
        // U = first k columns of the chosen side's eigenvectors (row-major n x n) -> n x k
        const double *Vs = c->V + (size_t)2 * i * kMaxEnvN * kMaxEnvN + (size_t)side * nmat * nmat;
        HIP_TRY(c, hipMemcpy2DAsync(c->U[i], sizeof(double) * d.k, Vs, sizeof(double) * nmat,
                                    sizeof(double) * d.k, nmat, hipMemcpyDeviceToDevice, c->stream));
        k_out[i] = d.k;
        c->Urows[q] = nmat;
        c->Ucols[q] = d.k;
    }
    return HOTRG_OK;
}

// Parity class tables of a Z2 block-form step (see ExpandParams): rows (and
// columns) (a, b, mu1, c) of the GEMM with the new labels of the transverse
// axes and the mu labels, inner K indices (b1', a2, c1', b2, c2) of a slice
// with the old labels (b1' counted in the slice parity when a slice fixes
// it).  Positions count each class in natural order.  Also fills the block
// sizes: R_g = N_g (pure T) or N_g + N_{1-g} + N_g (T | S_m | S_e).
int build_z2_tables(hotrg_ctx *c, int mu, const int tv[3], const int k[3], int Eb, int nA) {
    const int *D = c->dims;
    const int Da = D[tv[0]], Db = D[tv[1]], Dc = D[tv[2]], Dm = D[mu];
    const int ka = k[0], kb = k[1], kc = k[2];
    const auto &pa = c->new_par[tv[0]], &pb = c->new_par[tv[1]], &pc = c->new_par[tv[2]], &pm = c->par[mu];
    const auto &oa = c->par[tv[0]], &ob = c->par[tv[1]], &oc = c->par[tv[2]];
    if ((int)pa.size() != ka || (int)pb.size() != kb || (int)pc.size() != kc || (int)pm.size() != Dm ||
        (int)oa.size() != Da || (int)ob.size() != Db || (int)oc.size() != Dc)
        return set_err(HOTRG_EINVAL, "Z2 labels do not match the bond dimensions");
    auto &zl = c->z2l;
    const uint32_t M = (uint32_t)ka * kb * Dm * kc;
    auto &rt = c->rtab_h;
    rt.resize(M);
    uint32_t cnt[2] = {0, 0}, r = 0;
    for (int a = 0; a < ka; ++a)
        for (int b = 0; b < kb; ++b)
            for (int m = 0; m < Dm; ++m)
                for (int cc = 0; cc < kc; ++cc) {
                    const int p = pa[a] ^ pb[b] ^ pm[m] ^ pc[cc];
                    rt[r++] = (p ? Z2_PAR : 0u) | cnt[p]++;
                }
    // (the block form orders a slice's inner K indices as (b1', a2, c1', b2,
    // c2): a2 outside c1', so that both last products cover whole K runs per
    // (b1', a2), see contract())
    const uint32_t Ks = (uint32_t)Eb * Dc * Da * Db * Dc;
    auto &kt = c->ktab_h;
    kt.resize(Ks);
    uint32_t kcnt[2] = {0, 0}, kk = 0;
    for (int b1 = 0; b1 < Eb; ++b1)
        for (int a2 = 0; a2 < Da; ++a2)
            for (int c1 = 0; c1 < Dc; ++c1)
                for (int b2 = 0; b2 < Db; ++b2)
                    for (int c2 = 0; c2 < Dc; ++c2) {
                        const int p = (Eb == Db ? ob[b1] : 0) ^ oc[c1] ^ oa[a2] ^ ob[b2] ^ oc[c2];
                        kt[kk++] = (p ? Z2_PAR : 0u) | kcnt[p]++;
                    }
    for (int g = 0; g < 2; ++g) {
        zl.N[g] = cnt[g];
        zl.Kc[g] = kcnt[g];
        zl.R[g] = nA == 1 ? cnt[g] : M + cnt[g];
    }
    zl.coff[0] = 0;
    zl.coff[1] = (uint64_t)zl.R[0] * zl.N[0];
    if (zl.coff[1] + (uint64_t)zl.R[1] * zl.N[1] > 3 * (uint64_t)c->cap)
        return set_err(HOTRG_EINVAL, "Z2 output blocks exceed the output buffer");
    const size_t Dmax = (size_t)std::max(c->dcut, 2);
    if (!c->rtab) TRY(alloc_n(c, &c->rtab, Dmax * Dmax * Dmax * Dmax));
    if (!c->ktab) TRY(alloc_n(c, &c->ktab, Dmax * Dmax * Dmax * Dmax * Dmax));
    HIP_TRY(c, hipMemcpyAsync(c->rtab, rt.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->ktab, kt.data(), sizeof(uint32_t) * Ks, hipMemcpyHostToDevice, c->stream));
    c->z2_gen++;
    return HOTRG_OK;
}

// Tile form of the bf16 Z2 scatter (see ExpandParams): whether the thread
// dims of x are [nko K-outer | nro row | inner] with the K-outer dims a dense
// row-major walk over K groups of tnK indices, the row dims a dense walk over
// units of L1 rows, and the inner dims plus the second loop a dense run of
// tnK K indices, and the first loop one row per step.  Fills the tile fields
// (the slot table and the permuted isometry block `id` are rebuilt when the
// class tables changed) and returns false, so that the run form is used,
// when the layout does not match or a limit is exceeded.
int z2_tile_plan(hotrg_ctx *c, ExpandParams &p, const double *U, uint64_t threads, int nko, int nro, uint64_t Ks,
                 int id, const std::vector<uint8_t> *labs, const std::vector<uint32_t> &kt, bool *ok) {
    // (Ks: the natural row length, i.e. the number of columns; kt: the host
    // copy of the column table)
    *ok = false;
    if (id < 0 || id > 3 || nko < 0 || nro < 0 || nko + nro > p.nd || p.o1 != Ks || !labs) return HOTRG_OK;
    // parity labels of the summed index, the first and the second loop index
    if ((int)labs[0].size() != p.nsum || (int)labs[1].size() != p.L1 || (int)labs[2].size() != p.L2 ||
        p.nsum > 13 || p.L1 > 13 || p.L2 > 13)
        return HOTRG_OK;
    if (const char *e = getenv("HOTRG_Z2_TILE"))
        if (e[0] == '0') return HOTRG_OK;
    // inner dims and the second loop: a dense run [0, nK)
    std::vector<std::pair<uint64_t, uint64_t>> in;  // (stride, extent)
    uint64_t P = 1;
    for (int d = nko + nro; d < p.nd; ++d) {
        P *= p.ext[d].d;
        if (p.ext[d].d > 1) in.push_back({p.out_st[d], p.ext[d].d});
    }
    if (p.L2 > 1) in.push_back({p.o2, (uint64_t)p.L2});
    std::sort(in.begin(), in.end());
    uint64_t nK = 1;
    for (const auto &se : in) {
        if (se.first != nK) return HOTRG_OK;
        nK *= se.second;
    }
    // K-outer dims: groups K0 = kg nK, kg < Kg, Kg nK = Ks
    uint64_t st = nK, Kg = 1;
    for (int d = nko - 1; d >= 0; --d) {
        if (p.ext[d].d > 1 && p.out_st[d] != st) return HOTRG_OK;
        st *= p.ext[d].d;
        Kg *= p.ext[d].d;
    }
    if (st != Ks) return HOTRG_OK;
    // row dims: unit u starts at row u L1
    uint64_t rs = Ks * (uint64_t)p.L1, NRP = 1;
    for (int d = nko + nro - 1; d >= nko; --d) {
        if (p.ext[d].d > 1 && p.out_st[d] != rs) return HOTRG_OK;
        rs *= p.ext[d].d;
        NRP *= p.ext[d].d;
    }
    if (P == 0 || NRP * Kg * P != threads) return HOTRG_OK;
    if (kt.size() != Ks) return HOTRG_OK;
    // largest class share of one K group
    uint64_t maxnk = 0;
    for (uint64_t g = 0; g < Kg; ++g) {
        uint64_t n1 = 0;
        for (uint64_t k = g * nK; k < (g + 1) * nK; ++k) n1 += kt[k] >> 31;
        maxnk = std::max(maxnk, std::max(n1, nK - n1));
    }
    // slot table: inner threads by the class of their first K index in the
    // first K group (the class of every K index of a thread's run in any group
    // is that class xor a label of the loop index xor the group's parity, so
    // one parity per wave stays one parity in every group), each class padded
    // to whole waves
    if (c->tile_gen[id] != c->z2_gen) {
        std::vector<uint32_t> cls[2];
        for (uint64_t j = 0; j < P; ++j) {
            uint64_t rem = j, k0 = 0;
            for (int d = p.nd - 1; d >= nko + nro; --d) {
                k0 += (rem % p.ext[d].d) * p.out_st[d];
                rem /= p.ext[d].d;
            }
            cls[kt[k0] >> 31].push_back((uint32_t)j);
        }
        auto &tp = c->tperm_h[id];
        tp.clear();
        for (int q = 0; q < 2; ++q) {
            const size_t padded = (cls[q].size() + 63) / 64 * 64;
            tp.insert(tp.end(), cls[q].begin(), cls[q].end());
            tp.insert(tp.end(), padded - cls[q].size(), ~0u);
        }
        if (tp.size() > (size_t)Z2TILE_MAX_THREADS) return HOTRG_OK;
        c->tslots[id] = (uint32_t)tp.size();
        // summed indices by parity; the isometry block [l1][l2][j] over the
        // j-th summed index of parity lab1(l1) ^ lab2(l2) (the others meet
        // exact zeros of a one-sector column), NH entries, zero-padded
        std::vector<int> I[2];
        for (int i = 0; i < p.nsum; ++i) I[labs[0][i] & 1].push_back(i);
        const int NH = z2tile_nh(p.nsum, (int)std::max(I[0].size(), I[1].size()));
        for (int q = 0; q < 2; ++q) {
            c->tnI[id][q] = (uint32_t)I[q].size();
            c->tI[id][q] = 0;
            for (size_t j = 0; j < I[q].size(); ++j) c->tI[id][q] |= (uint64_t)I[q][j] << (4 * j);
        }
        c->tlab1[id] = c->tlab2[id] = 0;
        for (int l = 0; l < p.L1; ++l) c->tlab1[id] |= (uint32_t)(labs[1][l] & 1) << l;
        for (int l = 0; l < p.L2; ++l) c->tlab2[id] |= (uint32_t)(labs[2][l] & 1) << l;
        c->tNH[id] = NH;
        auto &ti = c->tidx_h[id];
        ti.assign((size_t)p.L1 * p.L2 * NH, -1);
        for (int l1 = 0; l1 < p.L1; ++l1)
            for (int l2 = 0; l2 < p.L2; ++l2) {
                const int need = (labs[1][l1] ^ labs[2][l2]) & 1;
                for (size_t j = 0; j < I[need].size() && (int)j < NH; ++j)
                    ti[((size_t)l1 * p.L2 + l2) * NH + j] =
                        (int32_t)((uint64_t)l1 * p.u1 + (uint64_t)l2 * p.u2 + (uint64_t)I[need][j] * p.us);
            }
        if (!c->tperm_d[id]) TRY(alloc_n(c, &c->tperm_d[id], (size_t)Z2TILE_MAX_THREADS));
        if (!c->tidx_d[id]) TRY(alloc_n(c, &c->tidx_d[id], (size_t)13 * 13 * 13));
        if (!c->tU_d[id]) TRY(alloc_n(c, &c->tU_d[id], (size_t)13 * 13 * 13));
        HIP_TRY(c, hipMemcpyAsync(c->tperm_d[id], tp.data(), sizeof(uint32_t) * tp.size(), hipMemcpyHostToDevice,
                                  c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->tidx_d[id], ti.data(), sizeof(int32_t) * ti.size(), hipMemcpyHostToDevice,
                                  c->stream));
        c->tile_gen[id] = c->z2_gen;
    }
    // the compacted isometry block (a tiny gather, every call: the A products
    // of T, S_m, S_e share the isometry, but it is cheap)
    launch_gather_or_zero(U, c->tidx_d[id], c->tU_d[id], (int)c->tidx_h[id].size(), c->stream);
    p.tslots = c->tslots[id];
    p.tperm = c->tperm_d[id];
    p.tU = c->tU_d[id];
    p.tNH = c->tNH[id];
    p.tlab1 = c->tlab1[id];
    p.tlab2 = c->tlab2[id];
    for (int q = 0; q < 2; ++q) {
        p.tI[q] = c->tI[id][q];
        p.tnI[q] = c->tnI[id][q];
    }
    p.tLD = (uint32_t)((maxnk + 7 + 7) / 8 * 8);
    p.tP = (uint32_t)P;
    p.tNRP = (uint32_t)NRP;
    p.tKg = (uint32_t)Kg;
    p.tnK = (uint32_t)nK;
    // units per tile: at most Z2TILE_MAX_THREADS threads and about 40 KB of tiles
    const uint64_t unit_bytes = (uint64_t)p.L1 * p.tLD * 4;
    uint64_t upb = std::min<uint64_t>(Z2TILE_MAX_THREADS / p.tslots, std::max<uint64_t>(1, 40960 / unit_bytes));
    p.tupb = (uint32_t)std::max<uint64_t>(1, std::min(upb, NRP));
    *ok = z2tile_lds_bytes(p) <= Z2TILE_MAX_LDS;
    return HOTRG_OK;
}

// Turns the last isometry product described by x into the Z2 block scatter
// (natural row length Ks, slice parity zs, tensor parity zP, first rows off[g]
// of the tensor in class g) into the blocks out / hi / lo, with host checks
// that every write stays inside its block.  For bf16 outputs whose thread
// dims are laid out as [nko K-outer | nro row | inner] (see z2_tile_plan) the
// tile form is used.
int z2_scatter(hotrg_ctx *c, XP &x, const double *U, uint64_t Ks, uint32_t zs, uint32_t zP, const uint32_t off[2],
               uint64_t rows_cap, bool mixed, double *const out[2], uint16_t *const hi[2], uint16_t *const lo[2],
               int nko = -1, int nro = -1, int tile_id = -1, const std::vector<uint8_t> *labs = nullptr) {
    ExpandParams &p = x.p;
    const auto &zl = c->z2l;
    if (p.nsum != p.L2 || p.L2 > 13 || (size_t)p.L1 * p.L2 * p.L2 * sizeof(double) > 48 * 1024)
        return set_err(HOTRG_EINVAL, "Z2 scatter: unsupported product shape");
    // rows of class g written: off[g] + (rows of parity zP ^ g); columns < Kc[b] <= ldk[b]
    for (int g = 0; g < 2; ++g)
        if ((uint64_t)off[g] + zl.N[zP ^ (uint32_t)g] > rows_cap)
            return set_err(HOTRG_EINVAL, "Z2 scatter rows out of bounds");
    if (Ks != (uint64_t)zl.Kc[0] + zl.Kc[1] || zl.ldk[0] < zl.Kc[0] || zl.ldk[1] < zl.Kc[1])
        return set_err(HOTRG_EINVAL, "Z2 scatter columns out of bounds");
    p.z2 = 1;
    // run form: every thread dim steps either whole rows (stride a multiple
    // of Ks) or K digits, the first loop steps whole rows, and the second
    // loop plus the K digits stay below Ks (no carry into the row part)
    {
        bool run = p.o1 % Ks == 0 && p.o1 / Ks < (1u << 20) && p.o2 < Ks;
        uint64_t kmax = (uint64_t)(p.L2 - 1) * p.o2;
        for (int d = 0; d < p.nd && run; ++d) {
            const uint64_t st = p.out_st[d], ext = p.ext[d].d;
            if (st % Ks == 0) continue;
            if (st >= Ks) run = false;
            kmax += (ext - 1) * st;
        }
        if (run && kmax < Ks) {
            p.z2 = 2;
            p.zrs = (uint32_t)(p.o1 / Ks);
            // pairs: the second loop walks adjacent K indices, and the hi / lo
            // blocks are 4-byte aligned
            p.zpair = mixed && p.o2 == 1 && ((uintptr_t)hi[0] & 3) == 0 && ((uintptr_t)hi[1] & 3) == 0 &&
                      ((uintptr_t)lo[0] & 3) == 0 && ((uintptr_t)lo[1] & 3) == 0;
        }
    }
    if (mixed && p.z2 == 2 && (((uintptr_t)hi[0] | (uintptr_t)hi[1] | (uintptr_t)lo[0] | (uintptr_t)lo[1]) & 15) == 0) {
        bool ok = false;
        TRY(z2_tile_plan(c, p, U, x.threads, nko, nro, Ks, tile_id, labs, c->ktab_h, &ok));
        if (ok) {
            p.z2 = 3;
            c->z2_tile_launches++;
        }
    }
    p.zld = make_fastdiv((uint32_t)Ks);
    p.rtab = c->rtab;
    p.ktab = c->ktab;
    p.zs = zs;
    p.zP = zP;
    p.zM = (uint32_t)c->rtab_h.size();
    for (int b = 0; b < 2; ++b) {
        p.zKc[b] = zl.Kc[b];
        p.zNr[b] = zl.N[b];
    }
    for (int b = 0; b < 2; ++b) {
        p.zrow_off[b] = off[b];
        p.zld_out[b] = (uint32_t)zl.ldk[b];
        p.zpkb[b] = (uint32_t)(zl.ldk[b] / PACK_K);
        p.zout[b] = mixed ? nullptr : out[b];
        p.zhi[b] = mixed ? hi[b] : nullptr;
        p.zlo[b] = mixed ? lo[b] : nullptr;
    }
    return HOTRG_OK;
}

// Contraction of one step with isometries c->U[0..2] (n_i x k_i, row-major).
int contract(hotrg_ctx *c, int mu, const int tv[3], const int k[3]) {
    const int *D = c->dims;
    uint64_t cst[8];
    canon_strides(D, cst);
    uint64_t lst[8];
    int ldim[8];
    for (int i = 0; i < 3; ++i) {
        lst[2 * i] = cst[2 * tv[i]];
        lst[2 * i + 1] = cst[2 * tv[i] + 1];
        ldim[2 * i] = ldim[2 * i + 1] = D[tv[i]];
    }
    lst[6] = cst[2 * mu];
    lst[7] = cst[2 * mu + 1];
    ldim[6] = ldim[7] = D[mu];
    const int Da = D[tv[0]], Db = D[tv[1]], Dc = D[tv[2]], Dm = D[mu];
    const int ka = k[0], kb = k[1], kc = k[2];
    const uint64_t M = (uint64_t)ka * kb * kc * Dm;  // rows of one tensor = columns
    const bool imp = c->cfg.impurities != 0;
    const bool se_pair = imp && c->n == 0;  // Eq. (2.8): S_e . S_e on the first step
    const int nA = imp ? 3 : 1;
    const int nA_shared = se_pair ? 2 : nA;  // operands multiplying B(T)
    const int nB = se_pair ? 2 : 1;
    if (M * M * 3 > c->cap * 3) return set_err(HOTRG_EINVAL, "new tensor exceeds capacity");
    const bool mixed = c->cfg.precision == HOTRG_BF16X3 && (c->n + 1) >= c->cfg.mixed_from_step;
    // K slices fix (alpha, a1') and, when a slice would exceed 2^31 elements
    // per tensor or the configured operand budget, also b1' (Eb = 1)
    auto slice_bytes = [&](uint64_t ks) {
        const uint64_t l = mixed ? (ks + 63) / 64 * 64 : ks;
        return mixed ? (uint64_t)4 * packed_rows(M) * l * (nA + nB) : (uint64_t)8 * M * l * (nA + nB);
    };
    const uint64_t Ks2 = (uint64_t)Db * Dc * Da * Db * Dc;
    const bool slice_b = M * (Ks2 + 63) >= (1ull << 31) ||
                         (c->cfg.slice_budget > 0 && slice_bytes(Ks2) > c->cfg.slice_budget);
    const int Eb = slice_b ? 1 : Db;  // b1' values inside one slice
    const uint64_t Ks = (uint64_t)Eb * Dc * Da * Db * Dc;
    if (M * (Ks + 63) >= (1ull << 31)) return set_err(HOTRG_ENOMEM, "operand slice exceeds 2^31 elements");
    // bf16 operand rows are padded with zero columns to a multiple of the
    // 64 k the kernel stages at a time
    const uint64_t ld = mixed ? (Ks + 63) / 64 * 64 : Ks;
    const uint64_t slice = M * ld;          // row-major operand slice of one tensor
    const uint64_t pslice = packed_rows(M) * ld;  // the same in the packed bf16 layout
    // when every A tensor multiplies the same B, their rows form one packed
    // block of nA * M rows (padded once, not per tensor) and one GEMM call
    const bool stack = mixed && nB == 1 && nA > 1;
    double *Asl = nullptr, *Bsl = nullptr;
    uint16_t *Ah = nullptr, *Al = nullptr, *Bh = nullptr, *Bl = nullptr;
    double *tail = nullptr;
    // Z2 block form: per parity class of the inner K index one operand block
    // pair (A rows of the GEMM class, B rows = columns of that class)
    const bool z2 = c->step_z2 && nB == 1;
    auto &zl = c->z2l;
    double *zA[2] = {nullptr, nullptr}, *zB[2] = {nullptr, nullptr};
    uint16_t *zAh[2] = {nullptr, nullptr}, *zAl[2] = {nullptr, nullptr};
    uint16_t *zBh[2] = {nullptr, nullptr}, *zBl[2] = {nullptr, nullptr};
    uint64_t z2_arows = 0, z2_brows = 0;  // rows allocated per A / B block
    if (z2) {
        TRY(build_z2_tables(c, mu, tv, k, Eb, nA));
        const uint32_t Nmax = std::max(zl.N[0], zl.N[1]);
        const uint64_t Amax = (uint64_t)std::max(zl.R[0], zl.R[1]);
        z2_arows = Amax;
        z2_brows = Nmax;
        uint64_t need = 0, offs[2][2];
        for (int b = 0; b < 2; ++b) {
            // bf16: whole packed k blocks; FP64: an even row length, so that
            // every row is 16-byte aligned for the DGEMM's vector loads
            zl.ldk[b] = mixed ? ((uint64_t)zl.Kc[b] + 63) / 64 * 64 : ((uint64_t)zl.Kc[b] + 1) / 2 * 2;
            const uint64_t ar = mixed ? packed_rows(Amax) : Amax, br = mixed ? packed_rows(Nmax) : Nmax;
            offs[b][0] = need;
            need += ar * zl.ldk[b];
            offs[b][1] = need;
            need += br * zl.ldk[b];
        }
        // (block offsets are 64-bit; the GEMMs take rows and k as int)
        if (Amax * zl.ldk[0] >= (1ull << 31) || Amax * zl.ldk[1] >= (1ull << 31))
            return set_err(HOTRG_ENOMEM, "Z2 operand block exceeds 2^31 elements");
        if (mixed) {
            TRY(ensure(c, c->z2_slices, sizeof(uint16_t) * 2 * need));
            TRY(ensure(c, c->gemm_tail, sizeof(double) * GEMM_TAIL_MAX_TILES * 256 * 256));
            tail = (double *)c->gemm_tail.p;
            uint16_t *base = (uint16_t *)c->z2_slices.p;
            for (int b = 0; b < 2; ++b) {
                zAh[b] = base + offs[b][0];
                zAl[b] = base + need + offs[b][0];
                zBh[b] = base + offs[b][1];
                zBl[b] = base + need + offs[b][1];
            }
            // padding columns (Kc .. ldk) are never written and must be zero
            if (zl.ldk[0] != zl.Kc[0] || zl.ldk[1] != zl.Kc[1])
                HIP_TRY(c, hipMemsetAsync(base, 0, sizeof(uint16_t) * 2 * need, c->stream));
        } else {
            TRY(ensure(c, c->z2_slices, sizeof(double) * need));
            double *base = (double *)c->z2_slices.p;
            for (int b = 0; b < 2; ++b) {
                zA[b] = base + offs[b][0];
                zB[b] = base + offs[b][1];
            }
        }
    } else if (mixed) {
        TRY(ensure(c, c->x3_slices, sizeof(uint16_t) * 2 * pslice * (nA + nB)));
        TRY(ensure(c, c->gemm_tail, sizeof(double) * GEMM_TAIL_MAX_TILES * 256 * 256));
        tail = (double *)c->gemm_tail.p;
        Ah = (uint16_t *)c->x3_slices.p;
        Al = Ah + pslice * nA;
        Bh = Al + pslice * nA;
        Bl = Bh + pslice * nB;
        // padding columns are never written by the products and must be zero;
        // padding rows only reach output rows / columns the GEMM drops
        if (ld != Ks) HIP_TRY(c, hipMemsetAsync(Ah, 0, sizeof(uint16_t) * 2 * pslice * (nA + nB), c->stream));
    } else {
        TRY(ensure(c, c->f64_slices, sizeof(double) * slice * (nA + nB)));
        Asl = (double *)c->f64_slices.p;
        Bsl = Asl + slice * nA;
    }
    double *Ua = c->U[0], *Ub = c->U[1], *Uc = c->U[2];
    const uint64_t usz[3] = {(uint64_t)Da * Da * ka, (uint64_t)Db * Db * kb, (uint64_t)Dc * Dc * kc};
    const uint64_t tsize = tensor_size(D);
    c->ev_used = 0;

    // Intermediate layouts (the index summed next is innermost, the GEMM row
    // part outermost in GEMM order, so every read is a contiguous run):
    //   Y1[a, mu1, b1', c1', a2, c1, b1]        Y2[a, b, mu1, b1', c1', a2, b2, c1]
    //   Z1[a', mu2', a2, b2, c2, c2', b2']      Z2[a', b', mu2', b1', a2, b2, c2, c2']
    // GEMM rows (a, b, mu1, c), columns (a', b', mu2', c'), K (b1', c1', a2, b2, c2);
    // b1' runs over Eb values (a slice may fix it).
    const int y1e[7] = {ka, Dm, Eb, Dc, Da, Dc, Db};
    uint64_t y1s[7];
    row_major_strides(7, y1e, y1s);
    const int y2e[8] = {ka, kb, Dm, Eb, Dc, Da, Db, Dc};
    uint64_t y2s[8];
    row_major_strides(8, y2e, y2s);
    const int z1e[7] = {ka, Dm, Da, Db, Dc, Dc, Db};
    uint64_t z1s[7];
    row_major_strides(7, z1e, z1s);
    const int z2e[8] = {ka, kb, Dm, Eb, Da, Db, Dc, Dc};
    uint64_t z2s[8];
    row_major_strides(8, z2e, z2s);

    // K-part strides of an operand row: (b1', c1', a2, b2, c2) in the dense
    // form, (b1', a2, c1', b2, c2) in the block form (the order of ktab); and
    // row strides
    const uint64_t kb1 = (uint64_t)Dc * Da * Db * Dc;
    const uint64_t kc1 = z2 ? (uint64_t)Db * Dc : (uint64_t)Da * Db * Dc;
    const uint64_t ka2 = z2 ? (uint64_t)Dc * Db * Dc : (uint64_t)Db * Dc;
    const uint64_t kb2 = Dc;
    // (the Z2 scatter splits natural offsets r Ks + k, so its row length is Ks)
    const uint64_t ldn = z2 ? Ks : ld;
    const uint64_t rs0 = (uint64_t)kb * Dm * kc * ldn, rs1 = (uint64_t)Dm * kc * ldn, rs2 = (uint64_t)kc * ldn;
    bool z2_init[2] = {false, false};
    // labels of the last products' summed index, first and second loop index:
    // old c, new c, old c (both products)
    const std::vector<uint8_t> tile_labs[3] = {c->par[tv[2]], c->new_par[tv[2]], c->par[tv[2]]};

    bool first_slice = true;
    const int nslices = Dm * Da * (Db / Eb);
    int sdone = 0;
    for (int g = 0; g < Dm; ++g) {       // alpha
      for (int f = 0; f < Da; ++f) {     // a1'
        for (int e0 = 0; e0 < Db; e0 += Eb) {  // first b1' of the slice
            // parity of the indices the slice fixes (alpha, a1', and b1' when Eb = 1)
            const uint32_t zs = z2 ? (uint32_t)(c->par[mu][g] ^ c->par[tv[0]][f] ^ (Eb == 1 ? c->par[tv[1]][e0] : 0))
                                   : 0u;
            // ---- A rows: T1 in {T, S_m, S_e}
            for (int t = 0; t < nA; ++t) {
                const uint64_t off = f * lst[1] + g * lst[7] + e0 * lst[3];
                const double *X1 = c->state[t] + off;
                {   // P1: Y1[a,mu1,b1',c1',a2,c1,b1] = sum_a1 Ua[(a1,a2),a] T1[a1,f,b1,b1',c1,c1',mu1,g]
                    XP x;
                    x.tdim(Dm, lst[6], y1s[1]);
                    x.tdim(Eb, lst[3], y1s[2]);
                    x.tdim(Dc, lst[5], y1s[3]);
                    x.tdim(Dc, lst[4], y1s[5]);
                    x.tdim(Db, lst[2], y1s[6]);
                    x.loops(ka, 1, y1s[0], Da, ka, y1s[4]);
                    x.sum(Da, lst[0], (uint64_t)Da * ka);
                    if (!x.fits(tsize - off, usz[0], c->cap)) return set_err(HOTRG_EINVAL, "P1 launch out of bounds");
                    launch_iso_expand(x.done(), X1, Ua, c->y1, nullptr, nullptr, c->stream);
                }
                {   // P2: Y2[a,b,mu1,b1',c1',a2,b2,c1] = sum_b1 Ub[(b1,b2),b] Y1
                    XP x;
                    x.tdim(ka, y1s[0], y2s[0]);
                    x.tdim(Dm, y1s[1], y2s[2]);
                    x.tdim(Eb, y1s[2], y2s[3]);
                    x.tdim(Dc, y1s[3], y2s[4]);
                    x.tdim(Da, y1s[4], y2s[5]);
                    x.tdim(Dc, y1s[5], y2s[7]);
                    x.loops(kb, 1, y2s[1], Db, kb, y2s[6]);
                    x.sum(Db, y1s[6], (uint64_t)Db * kb);
                    if (!x.fits(c->cap, usz[1], c->cap)) return set_err(HOTRG_EINVAL, "P2 launch out of bounds");
                    launch_iso_expand(x.done(), c->y1, Ub, c->y2, nullptr, nullptr, c->stream);
                }
                {   // P3: A[(a,b,mu1,c),(b1',c1',a2,b2,c2)] = sum_c1 Uc[(c1,c2),c] Y2
                    XP x;
                    if (z2) {  // tile layout: K-outer (b1', a2), rows (a, b, mu1), inner (c1', b2)
                        x.tdim(Eb, y2s[3], kb1);
                        x.tdim(Da, y2s[5], ka2);
                        x.tdim(ka, y2s[0], rs0);
                        x.tdim(kb, y2s[1], rs1);
                        x.tdim(Dm, y2s[2], rs2);
                        x.tdim(Dc, y2s[4], kc1);
                        x.tdim(Db, y2s[6], kb2);
                    } else {
                        x.tdim(ka, y2s[0], rs0);
                        x.tdim(kb, y2s[1], rs1);
                        x.tdim(Dm, y2s[2], rs2);
                        x.tdim(Eb, y2s[3], kb1);
                        x.tdim(Dc, y2s[4], kc1);
                        x.tdim(Da, y2s[5], ka2);
                        x.tdim(Db, y2s[6], kb2);
                    }
                    x.loops(kc, 1, ldn, Dc, kc, 1);
                    x.sum(Dc, y2s[7], (uint64_t)Dc * kc);
                    if (!x.fits(c->cap, usz[2], M * ldn)) return set_err(HOTRG_EINVAL, "P3 launch out of bounds");
                    if (z2) {
                        // A rows of tensor t in GEMM class g start at: T 0, S_m N_g, S_e M
                        uint32_t off[2];
                        for (int gg = 0; gg < 2; ++gg)
                            off[gg] = t == 0 ? 0u : (t == 1 ? zl.N[gg] : (uint32_t)M);
                        TRY(z2_scatter(c, x, Uc, Ks, zs, t == 1 ? 1u : 0u, off, z2_arows, mixed, zA, zAh, zAl, 2, 3,
                                       0, tile_labs));
                        launch_iso_expand(x.done(), c->y2, Uc, nullptr, nullptr, nullptr, c->stream);
                    } else if (mixed && stack) {  // rows t*M .. t*M + M - 1 of one packed block
                        x.packed(ld, (uint32_t)(t * M));
                        launch_iso_expand(x.done(), c->y2, Uc, nullptr, Ah, Al, c->stream);
                    } else if (mixed) {
                        x.packed(ld);
                        launch_iso_expand(x.done(), c->y2, Uc, nullptr, Ah + pslice * t, Al + pslice * t,
                                          c->stream);
                    } else
                        launch_iso_expand(x.done(), c->y2, Uc, Asl + slice * t, nullptr, nullptr, c->stream);
                }
            }
            // ---- B columns: T2 = T (and S_e for the first-step pair)
            for (int bidx = 0; bidx < nB; ++bidx) {
                const uint64_t off = g * lst[6];
                const double *X2 = c->state[bidx == 0 ? 0 : 2] + off;
                {   // Q1: Z1[a',mu2',a2,b2,c2,c2',b2'] = sum_a2' Ua[(f,a2'),a'] T2[a2,a2',b2,b2',c2,c2',g,mu2']
                    XP x;
                    x.tdim(Dm, lst[7], z1s[1]);
                    x.tdim(Da, lst[0], z1s[2]);
                    x.tdim(Db, lst[2], z1s[3]);
                    x.tdim(Dc, lst[4], z1s[4]);
                    x.tdim(Dc, lst[5], z1s[5]);
                    x.tdim(Db, lst[3], z1s[6]);
                    x.loops(ka, 1, z1s[0], 1, 0, 0);
                    x.sum(Da, lst[1], ka);
                    if (!x.fits(tsize - off, usz[0] - (uint64_t)f * Da * ka, c->cap))
                        return set_err(HOTRG_EINVAL, "Q1 launch out of bounds");
                    launch_iso_expand(x.done(), X2, Ua + (size_t)f * Da * ka, c->y1, nullptr, nullptr, c->stream);
                }
                {   // Q2: Z2[a',b',mu2',b1',a2,b2,c2,c2'] = sum_b2' Ub[(b1',b2'),b'] Z1
                    XP x;
                    x.tdim(ka, z1s[0], z2s[0]);
                    x.tdim(Dm, z1s[1], z2s[2]);
                    x.tdim(Da, z1s[2], z2s[4]);
                    x.tdim(Db, z1s[3], z2s[5]);
                    x.tdim(Dc, z1s[4], z2s[6]);
                    x.tdim(Dc, z1s[5], z2s[7]);
                    x.loops(kb, 1, z2s[1], Eb, (uint64_t)Db * kb, z2s[3]);
                    x.sum(Db, z1s[6], kb);
                    const uint64_t uoff = (uint64_t)e0 * Db * kb;  // rows (b1' = e0, b2') of Ub
                    if (!x.fits(c->cap, usz[1] - uoff, c->cap)) return set_err(HOTRG_EINVAL, "Q2 launch out of bounds");
                    launch_iso_expand(x.done(), c->y1, Ub + uoff, c->y2, nullptr, nullptr, c->stream);
                }
                {   // Q3: Bt[(a',b',mu2',c'),(b1',c1',a2,b2,c2)] = sum_c2' Uc[(c1',c2'),c'] Z2
                    XP x;
                    if (z2) {  // tile layout: K-outer (b1', a2), rows (a', b', mu2'), inner (b2, c2)
                        x.tdim(Eb, z2s[3], kb1);
                        x.tdim(Da, z2s[4], ka2);
                        x.tdim(ka, z2s[0], rs0);
                        x.tdim(kb, z2s[1], rs1);
                        x.tdim(Dm, z2s[2], rs2);
                    } else {
                        x.tdim(ka, z2s[0], rs0);
                        x.tdim(kb, z2s[1], rs1);
                        x.tdim(Dm, z2s[2], rs2);
                        x.tdim(Eb, z2s[3], kb1);
                        x.tdim(Da, z2s[4], ka2);
                    }
                    x.tdim(Db, z2s[5], kb2);
                    x.tdim(Dc, z2s[6], 1);
                    x.loops(kc, 1, ldn, Dc, (uint64_t)Dc * kc, kc1);
                    x.sum(Dc, z2s[7], kc);
                    if (!x.fits(c->cap, usz[2], M * ldn)) return set_err(HOTRG_EINVAL, "Q3 launch out of bounds");
                    if (z2) {
                        const uint32_t off[2] = {0u, 0u};
                        TRY(z2_scatter(c, x, Uc, Ks, zs, 0u, off, z2_brows, mixed, zB, zBh, zBl, 2, 3, 1, tile_labs));
                        launch_iso_expand(x.done(), c->y2, Uc, nullptr, nullptr, nullptr, c->stream);
                    } else if (mixed) {
                        x.packed(ld);
                        launch_iso_expand(x.done(), c->y2, Uc, nullptr, Bh + pslice * bidx, Bl + pslice * bidx,
                                          c->stream);
                    } else
                        launch_iso_expand(x.done(), c->y2, Uc, Bsl + slice * bidx, nullptr, nullptr, c->stream);
                }
            }
            // ---- GEMMs: C rows (+)= A B^T
            if (z2) {
                // block b (inner K parity b) feeds GEMM class g = b ^ zs:
                // C_g[R_g x N_g] (+)= A_b B_b^T over the Kc[b] indices of the
                // block; in mixed precision both products go in one launch
                X3Gemm xg[2];
                int nx = 0;
                double fl = 0;
                hipEvent_t e0 = next_event(c), e1 = next_event(c);
                if (e0) HIP_TRY(c, hipEventRecord(e0, c->stream));
                for (int b = 0; b < 2; ++b) {
                    const int gcls = b ^ (int)zs;
                    const uint32_t R = zl.R[gcls], N = zl.N[gcls], Kb = zl.Kc[b];
                    if (R == 0 || N == 0 || Kb == 0) continue;
                    double *Cg = c->cbuf + zl.coff[gcls];
                    const int acc = z2_init[gcls] ? 1 : 0;
                    z2_init[gcls] = true;
                    if (mixed)
                        xg[nx++] = X3Gemm{zAh[b], zAl[b], zBh[b], zBl[b], Cg, (int)R, 1, (int)N, (int)zl.ldk[b], N, acc};
                    else
                        launch_gemm_f64(zA[b], zB[b], Cg, (int)R, (int)N, (int)Kb, zl.ldk[b], zl.ldk[b], N, acc,
                                        c->stream);
                    fl += 2.0 * (double)R * (double)N * (double)Kb;
                }
                if (mixed && nx > 0) launch_gemm_bf16x3_multi(xg, nx, c->stream, tail);
                if (e1) HIP_TRY(c, hipEventRecord(e1, c->stream));
                c->gemm_launches++;
                c->gemm_flops += fl;
            }
            for (int bidx = 0; bidx < (z2 ? 0 : nB); ++bidx) {
                const int row0 = bidx == 0 ? 0 : 2;
                const int rows = bidx == 0 ? nA_shared : 1;
                hipEvent_t e0 = next_event(c), e1 = next_event(c);
                if (e0) HIP_TRY(c, hipEventRecord(e0, c->stream));
                double *Cp = c->cbuf + (size_t)row0 * M * M;
                if (mixed && stack)
                    launch_gemm_bf16x3(Ah, Al, Bh, Bl, Cp, (int)(M * rows), 1, (int)M, (int)ld, M,
                                       first_slice ? 0 : 1, c->stream, tail);
                else if (mixed)
                    launch_gemm_bf16x3(Ah + pslice * row0, Al + pslice * row0, Bh + pslice * bidx, Bl + pslice * bidx,
                                       Cp, (int)M, rows, (int)M, (int)ld, M, first_slice ? 0 : 1, c->stream, tail);
                else
                    launch_gemm_f64(Asl + slice * row0, Bsl + slice * bidx, Cp, (int)(M * rows), (int)M, (int)Ks, Ks,
                                    Ks, M, first_slice ? 0 : 1, c->stream);
                if (e1) HIP_TRY(c, hipEventRecord(e1, c->stream));
                c->gemm_launches++;
                c->gemm_flops += 2.0 * (double)(M * rows) * (double)M * (double)Ks;
            }
            first_slice = false;
            TRY(check_launch(c, "contraction slice"));
            TRY(report_progress(c, "contraction", c->n + 1, ++sdone, nslices));
        }
      }
    }
    if (z2)
        for (int gcls = 0; gcls < 2; ++gcls)
            if (!z2_init[gcls]) launch_zero(c->cbuf + zl.coff[gcls], (size_t)zl.R[gcls] * zl.N[gcls], c->stream);
    return HOTRG_OK;
}

// c_n = |C_T|_F; state <- perm(C)/c_n; ln Z bookkeeping.
int finish_step(hotrg_ctx *c, int mu, const int tv[3], const int k[3]) {
    int Dn[4];
    for (int q = 0; q < 4; ++q) Dn[q] = c->dims[q];
    for (int i = 0; i < 3; ++i) Dn[tv[i]] = k[i];
    const int Dm = c->dims[mu];
    const uint64_t M = (uint64_t)k[0] * k[1] * k[2] * Dm;
    const auto &zl = c->z2l;
    double ss = 0;
    if (c->step_z2) {
        // the T rows of both classes: the first N_g rows of C_g (row length N_g)
        double s2[2] = {0, 0};
        for (int g = 0; g < 2; ++g)
            launch_sumsq(c->cbuf + zl.coff[g], (size_t)zl.N[g] * zl.N[g], c->partials, 1024, c->scal + g, c->stream);
        HIP_TRY(c, hipMemcpyAsync(s2, c->scal, sizeof(s2), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        ss = s2[0] + s2[1];
    } else {
        launch_sumsq(c->cbuf, (size_t)(M * M), c->partials, 1024, c->scal, c->stream);
        HIP_TRY(c, hipMemcpyAsync(&ss, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    // accumulate GEMM event times of this step
    for (size_t e = 0; e + 1 < c->ev_used; e += 2) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, c->ev_pool[e], c->ev_pool[e + 1]) == hipSuccess) c->gemm_ms += ms;
    }
    c->ev_used = 0;
    double cn = std::sqrt(ss);
    if (!(cn > 0) || !std::isfinite(cn)) {
        c->failed = true;
        return set_err(HOTRG_ENUMERIC, "norm of the new tensor is not finite and positive at step " +
                                           std::to_string(c->n + 1));
    }
    // C row index ((a kb + b) Dm + mu1) kc + c, column likewise with primes
    const uint64_t cs_a = (uint64_t)k[1] * Dm * k[2], cs_b = (uint64_t)Dm * k[2], cs_m = k[2], cs_c = 1;
    const uint64_t rowst = M;
    int ext[8];
    uint32_t st[8];
    for (int q = 0; q < 4; ++q) {
        ext[2 * q] = ext[2 * q + 1] = Dn[q];
        uint64_t s;
        if (q == mu) s = cs_m;
        else s = (q == tv[0]) ? cs_a : (q == tv[1] ? cs_b : cs_c);
        st[2 * q] = (uint32_t)(s * rowst);
        st[2 * q + 1] = (uint32_t)s;
    }
    uint64_t mx = 0;
    PermParams pp = perm_params(8, ext, st, &mx);
    if (mx >= M * M || pp.total != M * M || M * M > c->cap)
        return set_err(HOTRG_EINVAL, "normalise / permute launch out of bounds");
    const int nt = c->cfg.impurities ? 3 : 1;
    if (c->step_z2) {
        // gather from the block form: row part of a canonical index from the
        // backward legs, column part from the forward legs
        Z2UnpackParams up{};
        up.nd = 8;
        up.total = (uint32_t)(M * M);
        for (int l = 0; l < 8; ++l) {
            up.ext[l] = make_fastdiv((uint32_t)ext[l]);
            const uint32_t sq = (l % 2 == 0) ? st[l] / (uint32_t)rowst : st[l];
            up.rst[l] = (l % 2 == 0) ? sq : 0u;
            up.cst[l] = (l % 2 == 0) ? 0u : sq;
        }
        up.rtab = c->rtab;
        for (int g = 0; g < 2; ++g) {
            up.C[g] = c->cbuf + zl.coff[g];
            up.N[g] = zl.N[g];
        }
        for (int t = 0; t < nt; ++t) {
            up.P = t == 1 ? 1u : 0u;
            for (int g = 0; g < 2; ++g) {
                up.row_off[g] = t == 0 ? 0u : (t == 1 ? zl.N[g] : (uint32_t)M);
                if ((uint64_t)up.row_off[g] + zl.N[up.P ^ (uint32_t)g] > zl.R[g])
                    return set_err(HOTRG_EINVAL, "Z2 unpack rows out of bounds");
            }
            launch_z2_unpack(up, c->state[t], 1.0 / cn, c->stream);
        }
    } else {
        for (int t = 0; t < nt; ++t)
            launch_permute(pp, c->cbuf + (size_t)t * M * M, c->state[t], 1.0 / cn, c->stream);
    }
    TRY(check_launch(c, "normalise / permute"));
    c->n += 1;
    c->last_cn = cn;
    c->lnz_acc += std::ldexp(std::log(cn), -c->n);
    for (int q = 0; q < 4; ++q) c->dims[q] = Dn[q];
    if (c->first_axis < 0) c->first_axis = mu;
    c->last_axis = mu;
    return HOTRG_OK;
}

void transverse_of(int mu, int tv[3]) {
    int j = 0;
    for (int q = 0; q < 4; ++q)
        if (q != mu) tv[j++] = q;
}

void free_checkpoint(hotrg_ctx *c, hotrg_ctx::Checkpoint &cp) {
    dev_free(c, cp.T);
    cp.T = nullptr;
    for (int i = 0; i < 3; ++i) {
        dev_free(c, cp.U[i]);
        dev_free(c, cp.lam[i]);
        dev_free(c, cp.V[i]);
        cp.U[i] = cp.lam[i] = cp.V[i] = nullptr;
    }
}

// Drops every stored checkpoint and returns its memory (waits for the stream,
// which may still read them).
int clear_checkpoints(hotrg_ctx *c) {
    if (c->ckpts.empty()) return HOTRG_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto &cp : c->ckpts) free_checkpoint(c, cp);
    c->ckpts.clear();
    return HOTRG_OK;
}

// Copy of everything the reverse pass needs from the step about to run: the
// state T, the isometries, and (for truncated axes) the chosen side's full
// eigendecomposition.  Isometries given by the caller count as constants.
// Built in c->pending; on failure the partial copy is freed again.
int save_checkpoint_into(hotrg_ctx *c, hotrg_ctx::Checkpoint &cp, int axis, const int tv[3], const int k[3],
                         bool given_u) {
    for (int q = 0; q < 4; ++q) cp.dims[q] = c->dims[q];
    cp.axis = axis;
    cp.z2 = c->step_z2;
    if (cp.z2) {
        for (int q = 0; q < 4; ++q) cp.par[q] = c->par[q];
        for (int i = 0; i < 3; ++i) cp.npar[i] = c->new_par[tv[i]];
    }
    const size_t ts = tensor_size(c->dims);
    TRY(alloc_n(c, &cp.T, ts));
    HIP_TRY(c, hipMemcpyAsync(cp.T, c->state[0], sizeof(double) * ts, hipMemcpyDeviceToDevice, c->stream));
    for (int i = 0; i < 3; ++i) {
        const int q = tv[i];
        const int nmat = c->dims[q] * c->dims[q];
        cp.tv[i] = q;
        cp.k[i] = k[i];
        cp.n[i] = nmat;
        cp.trunc[i] = !given_u && c->dec[q].truncated;
        cp.side[i] = cp.trunc[i] ? c->dec[q].side : 0;
        cp.flagged[i] = cp.trunc[i] && c->dec[q].flagged;
        TRY(alloc_n(c, &cp.U[i], (size_t)nmat * k[i]));
        HIP_TRY(c, hipMemcpyAsync(cp.U[i], c->U[i], sizeof(double) * nmat * k[i], hipMemcpyDeviceToDevice,
                                  c->stream));
        if (cp.trunc[i]) {
            const int side = c->dec[q].side;
            TRY(alloc_n(c, &cp.lam[i], (size_t)nmat));
            TRY(alloc_n(c, &cp.V[i], (size_t)nmat * nmat));
            HIP_TRY(c, hipMemcpyAsync(cp.lam[i], c->lam + (size_t)2 * i * kMaxEnvN + (size_t)side * nmat,
                                      sizeof(double) * nmat, hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(cp.V[i],
                                      c->V + (size_t)2 * i * kMaxEnvN * kMaxEnvN + (size_t)side * nmat * nmat,
                                      sizeof(double) * nmat * nmat, hipMemcpyDeviceToDevice, c->stream));
        }
    }
    return HOTRG_OK;
}

int save_checkpoint(hotrg_ctx *c, int axis, const int tv[3], const int k[3], bool given_u) {
    c->pending = hotrg_ctx::Checkpoint{};
    int rc = save_checkpoint_into(c, c->pending, axis, tv, k, given_u);
    if (rc != HOTRG_OK) {
        (void)hipStreamSynchronize(c->stream);
        free_checkpoint(c, c->pending);
    }
    return rc;
}

// Adds the phase intervals of the last completed step (waits for its end).
int flush_phases(hotrg_ctx *c) {
    if (!c->ph_pending) return HOTRG_OK;
    c->ph_pending = false;
    HIP_TRY(c, hipEventSynchronize(c->ph[3]));
    for (int i = 0; i < 3; ++i) {
        float ms = 0;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ph[i], c->ph[i + 1]));
        c->phase_ms[i] += ms;
    }
    c->phase_steps++;
    return HOTRG_OK;
}

// Parity of every isometry column (Z2 state only): the parity of the merged
// rows (i1, i2) it is non-zero on, p(i1) ^ p(i2).  *pure = false as soon as
// one column has non-zero rows of both parities (or none).
int z2_new_labels(hotrg_ctx *c, const int tv[3], const int k[3], const double *const *Uhost, bool *pure) {
    *pure = true;
    std::vector<double> U;
    for (int i = 0; i < 3; ++i) {
        const int q = tv[i], D = c->dims[q], n = D * D;
        const double *u;
        if (Uhost) {
            u = Uhost[q];
        } else {
            U.resize((size_t)n * k[i]);
            HIP_TRY(c, hipMemcpyAsync(U.data(), c->U[i], sizeof(double) * n * k[i], hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            u = U.data();
        }
        const auto &p = c->par[q];
        auto &np = c->new_par[q];
        np.assign(k[i], 0);
        for (int j = 0; j < k[i]; ++j) {
            int seen = 0;  // bit 0: an even row is non-zero, bit 1: an odd row
            for (int r = 0; r < n; ++r)
                if (u[(size_t)r * k[i] + j] != 0.0) seen |= 1 << (p[r / D] ^ p[r % D]);
            if (seen != 1 && seen != 2) {
                *pure = false;
                return HOTRG_OK;
            }
            np[j] = (uint8_t)(seen >> 1);
        }
    }
    return HOTRG_OK;
}

int run_step_body(hotrg_ctx *c, int axis, const int tv[3], const int k[3]) {
    HIP_TRY(c, hipEventRecord(c->ph[1], c->stream));
    TRY(contract(c, axis, tv, k));
    HIP_TRY(c, hipEventRecord(c->ph[2], c->stream));
    TRY(finish_step(c, axis, tv, k));
    HIP_TRY(c, hipEventRecord(c->ph[3], c->stream));
    c->ph_pending = true;
    return HOTRG_OK;
}

// Local leg numbering of a step along mu: 0..5 the transverse legs
// (a, a', b, b', c, c'), 6 = mu (backward), 7 = mu' (forward).
void local_legs(const int D[4], int mu, const int tv[3], uint64_t lst[8], int ldim[8]) {
    uint64_t cst[8];
    canon_strides(D, cst);
    for (int i = 0; i < 3; ++i) {
        lst[2 * i] = cst[2 * tv[i]];
        lst[2 * i + 1] = cst[2 * tv[i] + 1];
        ldim[2 * i] = ldim[2 * i + 1] = D[tv[i]];
    }
    lst[6] = cst[2 * mu];
    lst[7] = cst[2 * mu + 1];
    ldim[6] = ldim[7] = D[mu];
}

int do_step(hotrg_ctx *c, int axis, const double *const *Uhost, const int *khost) {
    if (!c) return set_err(HOTRG_EINVAL, "null context");
    if (c->failed) return set_err(HOTRG_ESTATE, "context is in a failed state");
    if (axis < 0 || axis > 3) return set_err(HOTRG_EINVAL, "axis must be 0..3");
    TRY(flush_phases(c));
    if (!c->ph[0])
        for (auto &e : c->ph) HIP_TRY(c, hipEventCreate(&e));
    HIP_TRY(c, hipEventRecord(c->ph[0], c->stream));
    int tv[3];
    transverse_of(axis, tv);
    uint64_t lst[8];
    int ldim[8];
    local_legs(c->dims, axis, tv, lst, ldim);
    int k[3];
    if (Uhost) {
        for (int i = 0; i < 3; ++i) {
            int q = tv[i];
            int nmat = c->dims[q] * c->dims[q];
            if (!Uhost[q] || khost[q] < 1 || khost[q] > std::max(c->dcut, 2) || khost[q] > nmat)
                return set_err(HOTRG_EINVAL, "isometry for a transverse axis missing or k out of range");
        }
        for (int q = 0; q < 4; ++q) c->dec[q] = Decision();
        c->iso_axis = axis;
        c->eig_sweeps = 0;
        c->eig_resid = 0;
        for (int i = 0; i < 3; ++i) {
            int q = tv[i];
            int nmat = c->dims[q] * c->dims[q];
            HIP_TRY(c, hipMemcpyAsync(c->U[i], Uhost[q], sizeof(double) * nmat * khost[q], hipMemcpyHostToDevice,
                                      c->stream));
            k[i] = khost[q];
            c->dec[q].k = k[i];
            c->Urows[q] = nmat;
            c->Ucols[q] = k[i];
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    } else {
        TRY(isometries(c, c->state[0], lst, ldim, tv, axis, k));
    }
    // Z2 labels of the new bonds; the block form needs them and a step that
    // is not the S_e . S_e pairing of the first step (Eq. (2.8))
    bool pure = false;
    if (c->z2) {
        int rz = z2_new_labels(c, tv, k, Uhost, &pure);
        if (rz != HOTRG_OK) {
            c->failed = true;
            return rz;
        }
    }
    c->step_z2 = pure && !c->cfg.dense_only && !(c->cfg.impurities && c->n == 0);
    int rc = c->cfg.keep_checkpoints ? save_checkpoint(c, axis, tv, k, Uhost != nullptr) : HOTRG_OK;
    if (rc != HOTRG_OK) {
        c->failed = true;
        return rc;
    }
    rc = run_step_body(c, axis, tv, k);
    if (rc == HOTRG_OK && c->z2) {
        if (pure)
            for (int i = 0; i < 3; ++i) c->par[tv[i]] = c->new_par[tv[i]];
        else
            c->z2 = false;
    }
    if (rc != HOTRG_OK) {
        // a failed step leaves the context failed; its checkpoint copy goes
        if (c->cfg.keep_checkpoints) {
            (void)hipStreamSynchronize(c->stream);
            free_checkpoint(c, c->pending);
        }
        c->failed = true;
        return rc;
    }
    if (c->cfg.keep_checkpoints) {
        c->pending.c = c->last_cn;
        c->ckpts.push_back(c->pending);
        c->pending = hotrg_ctx::Checkpoint{};
    }
    return HOTRG_OK;
}

int read_obs(hotrg_ctx *c, double *tr, double *trm, double *tre, std::vector<double> *A) {
    int axis = c->last_axis < 0 ? 3 : c->last_axis;
    const double *s1 = c->cfg.impurities ? c->state[1] : nullptr;
    const double *s2 = c->cfg.impurities ? c->state[2] : nullptr;
    launch_trace_obs(c->state[0], s1, s2, c->dims, axis, c->obs, c->stream);
    TRY(check_launch(c, "trace"));
    int Da = c->dims[axis];
    std::vector<double> h(3 + (size_t)Da * Da);
    HIP_TRY(c, hipMemcpyAsync(h.data(), c->obs, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *tr = h[0];
    *trm = h[1];
    *tre = h[2];
    if (A) A->assign(h.begin() + 3, h.end());
    return HOTRG_OK;
}

// ======================================================= reverse pass ====
// Work buffers of the reverse pass (grown on demand, kept for later calls).
enum {
    BW_TBAR0, BW_TBAR1, BW_CBAR, BW_CBART, BW_AT, BW_BT, BW_ABAR, BW_BBAR, BW_Z1, BW_Z2, BW_YB1, BW_YB2,
    BW_X3,   // packed bf16 hi / lo of C_bar, C_bar^T, A^T, B^T (mixed precision)
    BW_PART, // per-workgroup isometry-adjoint sums of the fused last-product adjoint
    BW_ZC,   // block form: packed bf16 hi / lo of the C_bar class blocks and their transposes
    BW_ZT,   // block form: transposed class operands A_b^T, B_b^T (FP64 or packed bf16 hi / lo)
    BW_ZO    // block form: class-block GEMM outputs A_bar_b, B_bar_b
};

template <typename T>
int bw_buf(hotrg_ctx *c, int which, size_t count, T **p) {
    TRY(ensure(c, c->bw[which], sizeof(T) * std::max<size_t>(count, 1)));
    *p = (T *)c->bw[which].p;
    return HOTRG_OK;
}

constexpr size_t kPartialCap = (size_t)1 << 20;  // doubles of split-sum partials

// A contraction whose every output index addresses only one operand, with
// few outputs and a long sum, as the outer-product reduction (RedParams);
// false when it does not have that form.
bool red_params(const EinsumParams &q, RedParams &r) {
    if (q.nout == 0 || q.nout > 4096 || q.S < 4096) return false;
    r = RedParams{};
    uint32_t Mo = 1, No = 1, xm1 = 0, yn1 = 0;
    for (int k = 0; k < q.ndo; ++k) {
        const uint32_t ext = q.oext[k].d;
        if (ext == 1) continue;
        if (q.ox[k] != 0 && q.oy[k] == 0) {
            if (r.ndm >= RED_MAXD) return false;
            r.mext[r.ndm] = ext;
            r.mx[r.ndm] = q.ox[k];
            r.mz[r.ndm] = q.oz[k];
            ++r.ndm;
            Mo *= ext;
            xm1 = q.ox[k];
        } else if (q.oy[k] != 0 && q.ox[k] == 0) {
            if (r.ndn >= RED_MAXD) return false;
            r.next[r.ndn] = ext;
            r.ny[r.ndn] = q.oy[k];
            r.nz[r.ndn] = q.oz[k];
            ++r.ndn;
            No *= ext;
            yn1 = q.oy[k];
        } else {
            return false;
        }
    }
    r.nds = q.nds;
    uint32_t sx1 = 0, sy1 = 0;
    for (int k = 0; k < q.nds; ++k) {
        r.sext[k] = make_fastdiv(q.sext[k]);
        r.sx[k] = q.sx[k];
        r.sy[k] = q.sy[k];
        if (q.sext[k] > 1) {
            sx1 = q.sx[k];
            sy1 = q.sy[k];
        }
    }
    r.mo = make_fastdiv(Mo);
    r.no = make_fastdiv(No);
    r.S = q.S;
    // stage each operand with its smaller-stride index fastest
    r.xmfast = Mo > 1 && (sx1 == 0 || xm1 < sx1);
    r.ynfast = No > 1 && (sy1 == 0 || yn1 < sy1);
    r.alpha = q.alpha;
    r.accumulate = q.accumulate;
    return true;
}

// A contraction with many outputs, a short sum (<= 100 terms) addressing both
// operands, and output indices that address only X (few) or only Y (many),
// as the small-matrix product (XmvParams); false otherwise.
bool xmv_params(const EinsumParams &q, XmvParams &r, bool *swap) {
    if (q.nout < (1u << 16) || q.S > 100 || q.S == 0) return false;
    // the small matrix is the operand whose own output indices span fewer values
    uint64_t px = 1, py = 1;
    for (int k = 0; k < q.ndo; ++k) {
        if (q.ox[k] != 0 && q.oy[k] == 0) px *= q.oext[k].d;
        if (q.oy[k] != 0 && q.ox[k] == 0) py *= q.oext[k].d;
    }
    *swap = py < px;
    const uint32_t *ox = *swap ? q.oy : q.ox, *oy = *swap ? q.ox : q.oy;
    const uint32_t *sx = *swap ? q.sy : q.sx, *sy = *swap ? q.sx : q.sy;
    r = XmvParams{};
    uint32_t M = 1, N = 1;
    for (int k = 0; k < q.ndo; ++k) {
        const uint32_t ext = q.oext[k].d;
        if (ext == 1) continue;
        if (ox[k] != 0 && oy[k] == 0) {
            if (r.ndm >= RED_MAXD) return false;
            r.mext[r.ndm] = ext;
            r.mx[r.ndm] = ox[k];
            r.mz[r.ndm] = q.oz[k];
            ++r.ndm;
            M *= ext;
        } else if (oy[k] != 0 && ox[k] == 0) {
            r.next[r.ndn] = q.oext[k];
            r.ny[r.ndn] = oy[k];
            r.nz[r.ndn] = q.oz[k];
            ++r.ndn;
            N *= ext;
        } else {
            return false;
        }
    }
    if (M > XMV_MAXM) return false;
    r.nds = q.nds;
    for (int k = 0; k < q.nds; ++k) {
        r.sext[k] = q.sext[k];
        r.sx[k] = sx[k];
        r.sy[k] = sy[k];
    }
    r.M = M;
    r.N = N;
    r.K = q.S;
    r.alpha = q.alpha;
    r.accumulate = q.accumulate;
    return true;
}

constexpr size_t kXmvCap = (size_t)XMV_MAXM * 100;  // doubles of the gathered small matrix

int run_einsum(hotrg_ctx *c, EP &e, const double *X, uint64_t xa, const double *Y, uint64_t ya, double *out,
               uint64_t za, double alpha, int accumulate, const char *what) {
    if (!e.fits(xa, ya, za)) return set_err(HOTRG_EINVAL, std::string(what) + ": launch out of bounds");
    const EinsumParams q = e.done(alpha, accumulate);
    RedParams r;
    XmvParams xv;
    if (red_params(q, r) && launch_red(r, X, Y, out, c->gram_part, kPartialCap, c->stream)) return check_launch(c, what);
    bool swap = false;
    if (xmv_params(q, xv, &swap)) {
        if (!c->xmv_buf) TRY(alloc_n(c, &c->xmv_buf, kXmvCap));
        if (launch_xmv(xv, swap ? Y : X, swap ? X : Y, out, c->xmv_buf, kXmvCap, c->stream))
            return check_launch(c, what);
    }
    launch_einsum(q, X, Y, out, c->gram_part, kPartialCap, c->stream);
    return check_launch(c, what);
}

// Fused adjoint of the last isometry product (output + isometry adjoint) when
// the sizes allow it; false -> the caller runs the two generic contractions.
int run_lastprod(hotrg_ctx *c, const LastProdParams &p, const double *X, uint64_t xa, const double *Y,
                 const double *U, uint64_t ua, double *out, uint64_t oa, double *Ubar, bool *done) {
    *done = false;
    const uint64_t xmax = (uint64_t)(p.n_o1 - 1) * p.x_o1 + (uint64_t)(p.n_o2 - 1) * p.x_o2 +
                          (uint64_t)(p.NJ - 1) * p.xj + (uint64_t)(p.L - 1) * p.xc + (uint64_t)(p.N - 1) * p.xs;
    const uint64_t omax = (uint64_t)(p.n_o1 - 1) * p.out_o1 + (uint64_t)(p.n_o2 - 1) * p.out_o2 +
                          (uint64_t)(p.NJ - 1) * p.oj + (uint64_t)(p.N - 1) * p.ol;
    const uint64_t umax = (uint64_t)(p.N - 1) * (p.ul + p.us) + (uint64_t)(p.L - 1) * p.uc;
    if (p.n_o1 == 0 || p.n_o2 == 0 || p.NJ == 0 || xmax >= xa || omax >= oa || umax >= ua || xmax >= (1ull << 32) ||
        omax >= (1ull << 32))
        return HOTRG_OK;
    if (p.cls) {
        // class-block source: natural offsets split as (o1 x_o1 + c xc) + (o2 x_o2 + j xj + s xs),
        // rows (multiples of ks) and K indices below ks
        const uint64_t ks = p.ks.d;
        const uint64_t kmax = (uint64_t)(p.n_o2 - 1) * p.x_o2 + (uint64_t)(p.NJ - 1) * p.xj + (uint64_t)(p.N - 1) * p.xs;
        if (ks == 0 || p.x_o1 % ks != 0 || p.xc % ks != 0 || kmax >= ks) return HOTRG_OK;
    }
    double *part;
    TRY(bw_buf(c, BW_PART, ((size_t)p.n_o1 * p.n_o2 + 64) * p.L * p.N * p.N, &part));
    if (!launch_lastprod_adjoint(p, X, Y, U, out, Ubar, part, c->stream)) return HOTRG_OK;
    *done = true;
    return check_launch(c, "last-product adjoint");
}

// Class tables of a checkpointed block-form step for its reverse pass (pure
// T): rows (a, b, mu1, c) with the new transverse labels and the mu labels,
// inner K indices of a slice in the dense order (b1', c1', a2, b2, c2) with
// the old labels (b1' in the slice parity when a slice fixes it); the rows of
// each class in class order (inv), and every row's and column's offset in
// Tbar (st: strides of (a, b, mu1, c) and (a', b', mu2', c') in Tbar).  The
// device tables c->rtab / c->ktab are overwritten (the next forward step
// rebuilds them).
int build_rev_z2(hotrg_ctx *c, const hotrg_ctx::Checkpoint &cp, int Eb, const uint32_t st[8], uint32_t N[2],
                 uint32_t Kc[2], uint32_t **inv, uint32_t **roff, uint32_t **coff) {
    const int *D = cp.dims;
    const int *tv = cp.tv, mu = cp.axis;
    const int Da = D[tv[0]], Db = D[tv[1]], Dc = D[tv[2]], Dm = D[mu];
    const int ka = cp.k[0], kb = cp.k[1], kc = cp.k[2];
    const auto &pa = cp.npar[0], &pb = cp.npar[1], &pc = cp.npar[2], &pm = cp.par[mu];
    const auto &oa = cp.par[tv[0]], &ob = cp.par[tv[1]], &oc = cp.par[tv[2]];
    if ((int)pa.size() != ka || (int)pb.size() != kb || (int)pc.size() != kc || (int)pm.size() != Dm ||
        (int)oa.size() != Da || (int)ob.size() != Db || (int)oc.size() != Dc)
        return set_err(HOTRG_EINVAL, "reverse pass: checkpoint Z2 labels do not match the bond dimensions");
    const uint32_t M = (uint32_t)ka * kb * Dm * kc;
    auto &rt = c->rtab_h;
    rt.resize(M);
    std::vector<uint32_t> hv((size_t)3 * M);  // inv | roff | coff
    uint32_t cnt[2] = {0, 0}, r = 0;
    std::vector<uint32_t> lists[2];
    for (int a = 0; a < ka; ++a)
        for (int b = 0; b < kb; ++b)
            for (int m = 0; m < Dm; ++m)
                for (int cc = 0; cc < kc; ++cc) {
                    const int p = pa[a] ^ pb[b] ^ pm[m] ^ pc[cc];
                    rt[r] = (p ? Z2_PAR : 0u) | cnt[p]++;
                    lists[p].push_back(r);
                    hv[M + r] = a * st[0] + b * st[1] + m * st[2] + cc * st[3];
                    hv[2 * (size_t)M + r] = a * st[4] + b * st[5] + m * st[6] + cc * st[7];
                    ++r;
                }
    std::copy(lists[0].begin(), lists[0].end(), hv.begin());
    std::copy(lists[1].begin(), lists[1].end(), hv.begin() + lists[0].size());
    const uint32_t Ks = (uint32_t)Eb * Dc * Da * Db * Dc;
    auto &kt = c->ktab_h;
    kt.resize(Ks);
    uint32_t kcnt[2] = {0, 0}, kk = 0;
    for (int b1 = 0; b1 < Eb; ++b1)
        for (int c1 = 0; c1 < Dc; ++c1)
            for (int a2 = 0; a2 < Da; ++a2)
                for (int b2 = 0; b2 < Db; ++b2)
                    for (int c2 = 0; c2 < Dc; ++c2) {
                        const int p = (Eb == Db ? ob[b1] : 0) ^ oc[c1] ^ oa[a2] ^ ob[b2] ^ oc[c2];
                        kt[kk++] = (p ? Z2_PAR : 0u) | kcnt[p]++;
                    }
    for (int g = 0; g < 2; ++g) {
        N[g] = cnt[g];
        Kc[g] = kcnt[g];
    }
    // the transposed B operand orders its K indices (b1', a2, b2, c2, c1') (its
    // product steps c1'); kmapq lists those entries by dense index
    auto &kq = c->ktabq_h;
    auto &km = c->kmapq_h;
    kq.resize(Ks);
    km.resize(Ks);
    {
        uint32_t qc[2] = {0, 0}, kk2 = 0;
        for (int b1 = 0; b1 < Eb; ++b1)
            for (int a2 = 0; a2 < Da; ++a2)
                for (int b2 = 0; b2 < Db; ++b2)
                    for (int c2 = 0; c2 < Dc; ++c2)
                        for (int c1 = 0; c1 < Dc; ++c1) {
                            const int p = (Eb == Db ? ob[b1] : 0) ^ oc[c1] ^ oa[a2] ^ ob[b2] ^ oc[c2];
                            const uint32_t e = (p ? Z2_PAR : 0u) | qc[p]++;
                            kq[kk2++] = e;
                            km[(((size_t)b1 * Dc + c1) * Da + a2) * Db * Dc + (size_t)b2 * Dc + c2] = e;
                        }
    }
    const size_t Dmax = (size_t)std::max(c->dcut, 2);
    if (!c->rtab) TRY(alloc_n(c, &c->rtab, Dmax * Dmax * Dmax * Dmax));
    if (!c->ktab) TRY(alloc_n(c, &c->ktab, Dmax * Dmax * Dmax * Dmax * Dmax));
    if (!c->ktabq) TRY(alloc_n(c, &c->ktabq, Dmax * Dmax * Dmax * Dmax * Dmax));
    if (!c->kmapq) TRY(alloc_n(c, &c->kmapq, Dmax * Dmax * Dmax * Dmax * Dmax));
    if (!c->rev_tabs) TRY(alloc_n(c, &c->rev_tabs, 3 * Dmax * Dmax * Dmax * Dmax));
    HIP_TRY(c, hipMemcpyAsync(c->ktabq, kq.data(), sizeof(uint32_t) * Ks, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->kmapq, km.data(), sizeof(uint32_t) * Ks, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->rtab, rt.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->ktab, kt.data(), sizeof(uint32_t) * Ks, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->rev_tabs, hv.data(), sizeof(uint32_t) * hv.size(), hipMemcpyHostToDevice,
                              c->stream));
    // the host vectors must outlive the copies
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->z2_gen++;
    *inv = c->rev_tabs;
    *roff = c->rev_tabs + M;
    *coff = c->rev_tabs + 2 * (size_t)M;
    return HOTRG_OK;
}

// Transposed block scatter of a reverse-pass operand product (natural offset
// o = K M + r; rows = inner K indices in the order of the row table ktab_d,
// columns = GEMM rows r): block b gets rows K_b, row length ld[b ^ zs].
// bf16 outputs use the tile form of the forward scatter with the roles of the
// tables exchanged (rows = K, columns = r) when x's thread dims are laid out
// [nko column-outer | nro K-row | column-inner] with the first loop stepping
// one K row and the second a column run (labs: labels of the summed index,
// the first and the second loop index); otherwise the loops are exchanged back
// and the element scatter runs, after checks that the thread dims split into
// K digits (strides multiples of M) and row digits (strides below M) without
// carries.
int z2t_scatter(hotrg_ctx *c, XP &x, const double *U, uint64_t M, uint64_t Ks, uint32_t zs, const uint32_t N[2],
                const uint32_t Kc[2], const uint64_t ld[2], bool mixed, double *const out[2], uint16_t *const hi[2],
                uint16_t *const lo[2], const uint32_t *ktab_d, int tile_id, int nko, int nro,
                const std::vector<uint8_t> *labs) {
    ExpandParams &p = x.p;
    for (int b = 0; b < 2; ++b)
        if (ld[b ^ zs] < N[b ^ zs]) return set_err(HOTRG_EINVAL, "reverse Z2 scatter: block row too short");
    (void)Kc;
    p.zld = make_fastdiv((uint32_t)M);
    p.zs = zs;
    p.zP = 0;
    // (the tile kernel needs the column run loop as long as the summed index)
    if (mixed && tile_id >= 2 && p.o1 == M && p.nsum == p.L2 && p.L1 <= 13 &&
        (((uintptr_t)hi[0] | (uintptr_t)hi[1] | (uintptr_t)lo[0] | (uintptr_t)lo[1]) & 15) == 0) {
        // rows: K (row table ktab_d, Kc per class); columns: r (rtab, N per class);
        // the kernel's block b (columns of class b) is our block b ^ zs
        p.rtab = ktab_d;
        p.ktab = c->rtab;
        p.zM = (uint32_t)Ks;
        for (int b = 0; b < 2; ++b) {
            p.zNr[b] = Kc[b];
            p.zKc[b] = N[b];
            p.zrow_off[b] = 0;
            p.zld_out[b] = (uint32_t)ld[b];
            p.zpkb[b] = (uint32_t)(ld[b] / PACK_K);
            p.zout[b] = nullptr;
            p.zhi[b] = hi[b ^ zs];
            p.zlo[b] = lo[b ^ zs];
        }
        bool ok = false;
        TRY(z2_tile_plan(c, p, U, x.threads, nko, nro, M, tile_id, labs, c->rtab_h, &ok));
        if (ok) {
            p.z2 = 3;
            c->z2_tile_launches++;
            return HOTRG_OK;
        }
    }
    if (p.o1 == M) {  // back to (column step, K step) loops for the element scatter
        std::swap(p.L1, p.L2);
        std::swap(p.u1, p.u2);
        std::swap(p.o1, p.o2);
    }
    if (p.nsum != p.L2 || p.L2 > 13 || (size_t)p.L1 * p.L2 * p.L2 * sizeof(double) > 48 * 1024)
        return set_err(HOTRG_EINVAL, "reverse Z2 scatter: unsupported product shape");
    if (p.o1 >= M || p.o2 % M != 0) return set_err(HOTRG_EINVAL, "reverse Z2 scatter: unsupported loop strides");
    uint64_t rmax = (uint64_t)(p.L1 - 1) * p.o1, kmax = (uint64_t)(p.L2 - 1) * (p.o2 / M);
    for (int d = 0; d < p.nd; ++d) {
        const uint64_t stv = p.out_st[d], ext = p.ext[d].d;
        if (stv % M == 0) kmax += (ext - 1) * (stv / M);
        else if (stv < M) rmax += (ext - 1) * stv;
        else return set_err(HOTRG_EINVAL, "reverse Z2 scatter: a thread dim mixes rows and K");
    }
    if (rmax >= M || kmax >= Ks) return set_err(HOTRG_EINVAL, "reverse Z2 scatter: launch out of bounds");
    p.z2 = 4;
    p.zrs = (uint32_t)(p.o2 / M);
    p.rtab = c->rtab;
    p.ktab = ktab_d;
    for (int b = 0; b < 2; ++b) {
        const uint32_t g = (uint32_t)b ^ zs;
        p.zrow_off[b] = 0;
        p.zld_out[b] = (uint32_t)ld[g];
        p.zpkb[b] = (uint32_t)(ld[g] / PACK_K);
        p.zout[b] = mixed ? nullptr : out[b];
        p.zhi[b] = mixed ? hi[b] : nullptr;
        p.zlo[b] = mixed ? lo[b] : nullptr;
    }
    return HOTRG_OK;
}

// Tbar_prev (dims of the checkpoint) = adjoint of one step applied to Tbar
// (dims after the step).  c_n is a constant (reading R5), so
// C_bar = perm^-1(Tbar) / c_n, then C = sum_s A_s B_s^T gives
// A_bar_s = C_bar B_s and B_bar_s = C_bar^T A_s, which flow back through the
// isometry products into T and the isometries; the isometries flow back
// through the eigendecomposition and the environments into T.
int backward_step(hotrg_ctx *c, const hotrg_ctx::Checkpoint &cp, const double *Tbar, double *Tprev, bool mixed,
                  int step) {
    const int *D = cp.dims;
    const int mu = cp.axis;
    const int *tv = cp.tv;
    uint64_t cst[8];
    canon_strides(D, cst);
    uint64_t lst[8];
    int ldim[8];
    for (int i = 0; i < 3; ++i) {
        lst[2 * i] = cst[2 * tv[i]];
        lst[2 * i + 1] = cst[2 * tv[i] + 1];
        ldim[2 * i] = ldim[2 * i + 1] = D[tv[i]];
    }
    lst[6] = cst[2 * mu];
    lst[7] = cst[2 * mu + 1];
    ldim[6] = ldim[7] = D[mu];
    const int Da = D[tv[0]], Db = D[tv[1]], Dc = D[tv[2]], Dm = D[mu];
    const int ka = cp.k[0], kb = cp.k[1], kc = cp.k[2];
    const uint64_t M = (uint64_t)ka * kb * Dm * kc;  // rows = columns of C
    // K slices as in the forward: (alpha, a1') fixed, and b1' too (Eb = 1)
    // where a two-index slice exceeds 2^31 elements or the operand budget
    const uint64_t Ks2 = (uint64_t)Db * Dc * Da * Db * Dc;
    const bool slice_b = M * Ks2 >= (1ull << 31) ||
                         (c->cfg.slice_budget > 0 && (uint64_t)4 * 8 * M * Ks2 > c->cfg.slice_budget);
    const int Eb = slice_b ? 1 : Db;
    const uint64_t Ks = (uint64_t)Eb * Dc * Da * Db * Dc;
    const uint64_t tsize = tensor_size(D);
    const double *T = cp.T;
    const double *Ua = cp.U[0], *Ub = cp.U[1], *Uc = cp.U[2];
    const uint64_t usz[3] = {(uint64_t)Da * Da * ka, (uint64_t)Db * Db * kb, (uint64_t)Dc * Dc * kc};
    if (M * Ks >= (1ull << 31) || M * M >= (1ull << 31))
        return set_err(HOTRG_ENOMEM, "reverse pass: operand slice exceeds 2^31 elements");

    // Z2 block form (the forward step ran in it): the reverse GEMMs split per
    // parity class like the forward's, A_bar_b = C_bar_g B_b, B_bar_b =
    // C_bar_g^T A_b (g = b ^ slice parity), on class blocks built from the
    // checkpoint's labels; their outputs go back to the natural layout (exact
    // zeros elsewhere) for the adjoint contractions below
    const bool z2 = cp.z2;
    uint32_t zN[2] = {0, 0}, zKc[2] = {0, 0};  // rows (= columns) and inner K indices per class
    uint64_t zld[2] = {0, 0};                  // k-dim row length of class g's operands
    uint16_t *zCh[2] = {}, *zCl[2] = {}, *zCTh[2] = {}, *zCTl[2] = {};
    uint16_t *zATh[2] = {}, *zATl[2] = {}, *zBTh[2] = {}, *zBTl[2] = {};
    double *zAT[2] = {}, *zBT[2] = {}, *zAo[2] = {}, *zBo[2] = {};
    double *Cbar, *CbarT, *AT = nullptr, *BT = nullptr, *Abar, *Bbar, *Z1, *Z2, *Yb1, *Yb2;
    TRY(bw_buf(c, BW_CBAR, M * M, &Cbar));
    TRY(bw_buf(c, BW_CBART, M * M, &CbarT));
    // mixed precision: the reverse GEMMs run as bf16x3 products on packed
    // operands with row length ldM (the recomputed A^T, B^T go there directly)
    // (block form: the transposed operands' natural offsets K M + r are split by the scatter)
    const uint64_t ldM = mixed && !z2 ? (M + 63) / 64 * 64 : M;  // row length of A^T, B^T (and C_bar splits)
    const uint64_t pC = packed_rows(M) * ldM, pK = packed_rows(Ks) * ldM;
    uint16_t *Ch = nullptr, *Cl = nullptr, *CTh = nullptr, *CTl = nullptr;
    uint16_t *ATh = nullptr, *ATl = nullptr, *BTh = nullptr, *BTl = nullptr;
    double *tail = nullptr;
    if (mixed && z2) {
        TRY(ensure(c, c->gemm_tail, sizeof(double) * GEMM_TAIL_MAX_TILES * 256 * 256));
        tail = (double *)c->gemm_tail.p;
    } else if (mixed) {
        if (M * ldM >= (1ull << 32) || Ks * ldM >= (1ull << 31))
            return set_err(HOTRG_ENOMEM, "reverse pass: packed operand exceeds 2^31 elements");
        TRY(ensure(c, c->gemm_tail, sizeof(double) * GEMM_TAIL_MAX_TILES * 256 * 256));
        tail = (double *)c->gemm_tail.p;
        uint16_t *x3;
        TRY(bw_buf(c, BW_X3, 4 * pC + 4 * pK, &x3));
        Ch = x3;
        Cl = Ch + pC;
        CTh = Cl + pC;
        CTl = CTh + pC;
        ATh = CTl + pC;
        ATl = ATh + pK;
        BTh = ATl + pK;
        BTl = BTh + pK;
        // padding columns of A^T, B^T are never written by the products
        if (ldM != M) HIP_TRY(c, hipMemsetAsync(ATh, 0, sizeof(uint16_t) * 4 * pK, c->stream));
    } else if (!z2) {
        TRY(bw_buf(c, BW_AT, M * Ks, &AT));
        TRY(bw_buf(c, BW_BT, M * Ks, &BT));
    }
    TRY(bw_buf(c, BW_ABAR, M * Ks, &Abar));
    TRY(bw_buf(c, BW_BBAR, M * Ks, &Bbar));
    TRY(bw_buf(c, BW_Z1, c->cap, &Z1));
    TRY(bw_buf(c, BW_Z2, c->cap, &Z2));
    TRY(bw_buf(c, BW_YB1, c->cap, &Yb1));
    TRY(bw_buf(c, BW_YB2, c->cap, &Yb2));
    double *Y1 = c->y1, *Y2 = c->y2;
    double *Ubar[3];  // in the forward's eigenvector scratch, free during the reverse pass
    for (int i = 0; i < 3; ++i) Ubar[i] = c->V + (size_t)i * kMaxEnvN * kMaxEnvN;
    for (int i = 0; i < 3; ++i) launch_zero(Ubar[i], usz[i], c->stream);
    launch_zero(Tprev, tsize, c->stream);

    // C_bar and its transpose from Tbar (new dims: k on transverse axes, Dm on mu)
    {
        int Dn[4];
        for (int q = 0; q < 4; ++q) Dn[q] = D[q];
        for (int i = 0; i < 3; ++i) Dn[tv[i]] = cp.k[i];
        uint64_t ncs[8];
        canon_strides(Dn, ncs);
        const int ext[8] = {ka, kb, Dm, kc, ka, kb, Dm, kc};
        uint32_t st[8] = {(uint32_t)ncs[2 * tv[0]], (uint32_t)ncs[2 * tv[1]], (uint32_t)ncs[2 * mu],
                          (uint32_t)ncs[2 * tv[2]], (uint32_t)ncs[2 * tv[0] + 1], (uint32_t)ncs[2 * tv[1] + 1],
                          (uint32_t)ncs[2 * mu + 1], (uint32_t)ncs[2 * tv[2] + 1]};
        uint64_t mx;
        PermParams pp = perm_params(8, ext, st, &mx);
        if (mx >= M * M) return set_err(HOTRG_EINVAL, "C_bar launch out of bounds");
        if (z2) {
            uint32_t *inv, *roff, *coff;
            TRY(build_rev_z2(c, cp, Eb, st, zN, zKc, &inv, &roff, &coff));
            c->z2_rev_steps++;
            launch_z2_cbar(Tbar, inv, roff, coff, zN[0], zN[1], 1.0 / cp.c, Cbar, CbarT, c->stream);
            TRY(check_launch(c, "C_bar class blocks"));
        }
    }
    if (z2) {
        // class buffers: C_bar_g (and transposes) packed for the bf16x3 GEMMs,
        // transposed class operands (rows K_b, row length zld[g]), GEMM outputs
        const uint32_t Nmax = std::max(zN[0], zN[1]);
        for (int g = 0; g < 2; ++g) zld[g] = mixed ? ((uint64_t)zN[g] + 63) / 64 * 64 : ((uint64_t)zN[g] + 1) / 2 * 2;
        const uint64_t ldmax = std::max<uint64_t>(std::max(zld[0], zld[1]), 1);
        if ((uint64_t)Nmax * ldmax >= (1ull << 31) || (uint64_t)std::max(zKc[0], zKc[1]) * ldmax >= (1ull << 31))
            return set_err(HOTRG_ENOMEM, "reverse pass: class operand exceeds 2^31 elements");
        if (mixed) {
            uint64_t cpk[2], need = 0;
            for (int g = 0; g < 2; ++g) {
                cpk[g] = packed_rows(zN[g]) * zld[g];
                need += cpk[g];
            }
            uint16_t *zc;
            TRY(bw_buf(c, BW_ZC, 4 * need, &zc));
            uint64_t o = 0;
            for (int g = 0; g < 2; ++g) {
                zCh[g] = zc + o;
                zCl[g] = zc + need + o;
                zCTh[g] = zc + 2 * need + o;
                zCTl[g] = zc + 3 * need + o;
                o += cpk[g];
            }
            const uint64_t sq0 = (uint64_t)zN[0] * zN[0];
            for (int g = 0; g < 2; ++g) {
                if (zN[g] == 0) continue;
                launch_split_pack(Cbar + (g ? sq0 : 0), zN[g], zN[g], (uint32_t)zld[g], zCh[g], zCl[g], c->stream);
                launch_split_pack(CbarT + (g ? sq0 : 0), zN[g], zN[g], (uint32_t)zld[g], zCTh[g], zCTl[g],
                                  c->stream);
            }
            uint64_t tpk[2], tneed = 0;
            for (int b = 0; b < 2; ++b) {
                tpk[b] = packed_rows(zKc[b]) * ldmax;
                tneed += tpk[b];
            }
            uint16_t *zt;
            TRY(bw_buf(c, BW_ZT, 4 * tneed, &zt));
            // padding columns of a block are never written in a slice whose
            // class row is shorter; they meet zero padding of C_bar, but must
            // hold finite values
            HIP_TRY(c, hipMemsetAsync(zt, 0, sizeof(uint16_t) * 4 * tneed, c->stream));
            for (int b = 0; b < 2; ++b) {
                const uint64_t o2 = b ? tpk[0] : 0;
                zATh[b] = zt + o2;
                zATl[b] = zt + tneed + o2;
                zBTh[b] = zt + 2 * tneed + o2;
                zBTl[b] = zt + 3 * tneed + o2;
            }
        } else {
            double *zt;
            TRY(bw_buf(c, BW_ZT, 2 * (uint64_t)Ks * ldmax, &zt));
            zAT[0] = zt;
            zAT[1] = zt + (uint64_t)zKc[0] * ldmax;
            zBT[0] = zt + (uint64_t)Ks * ldmax;
            zBT[1] = zBT[0] + (uint64_t)zKc[0] * ldmax;
        }
        double *zo;
        TRY(bw_buf(c, BW_ZO, 2 * (uint64_t)Nmax * Ks, &zo));
        zAo[0] = zo;
        zAo[1] = zo + (uint64_t)Nmax * zKc[0];
        zBo[0] = zo + (uint64_t)Nmax * Ks;
        zBo[1] = zBo[0] + (uint64_t)Nmax * zKc[0];
        TRY(check_launch(c, "C_bar class splits"));
    } else {
        const int ext[8] = {ka, kb, Dm, kc, ka, kb, Dm, kc};
        int Dn[4];
        for (int q = 0; q < 4; ++q) Dn[q] = D[q];
        for (int i = 0; i < 3; ++i) Dn[tv[i]] = cp.k[i];
        uint64_t ncs[8];
        canon_strides(Dn, ncs);
        uint32_t st[8] = {(uint32_t)ncs[2 * tv[0]], (uint32_t)ncs[2 * tv[1]], (uint32_t)ncs[2 * mu],
                          (uint32_t)ncs[2 * tv[2]], (uint32_t)ncs[2 * tv[0] + 1], (uint32_t)ncs[2 * tv[1] + 1],
                          (uint32_t)ncs[2 * mu + 1], (uint32_t)ncs[2 * tv[2] + 1]};
        uint64_t mx;
        PermParams pp = perm_params(8, ext, st, &mx);
        launch_permute(pp, Tbar, Cbar, 1.0 / cp.c, c->stream);
        uint32_t stT[8] = {st[4], st[5], st[6], st[7], st[0], st[1], st[2], st[3]};
        pp = perm_params(8, ext, stT, &mx);
        launch_permute(pp, Tbar, CbarT, 1.0 / cp.c, c->stream);
        if (mixed) {
            launch_split_pack(Cbar, (uint32_t)M, (uint32_t)M, (uint32_t)ldM, Ch, Cl, c->stream);
            launch_split_pack(CbarT, (uint32_t)M, (uint32_t)M, (uint32_t)ldM, CTh, CTl, c->stream);
        }
        TRY(check_launch(c, "C_bar"));
    }

    const int y1e[7] = {ka, Dm, Eb, Dc, Da, Dc, Db};
    uint64_t y1s[7];
    row_major_strides(7, y1e, y1s);
    const int y2e[8] = {ka, kb, Dm, Eb, Dc, Da, Db, Dc};
    uint64_t y2s[8];
    row_major_strides(8, y2e, y2s);
    const int z1e[7] = {ka, Dm, Da, Db, Dc, Dc, Db};
    uint64_t z1s[7];
    row_major_strides(7, z1e, z1s);
    const int z2e[8] = {ka, kb, Dm, Eb, Da, Db, Dc, Dc};
    uint64_t z2s[8];
    row_major_strides(8, z2e, z2s);
    const uint64_t ks0 = (uint64_t)Dc * Da * Db * Dc, ks1 = (uint64_t)Da * Db * Dc, ks2 = (uint64_t)Db * Dc,
                   ks3 = Dc;
    // row-index strides of (a, b, mu1, c) in C / the operands
    const uint64_t r0 = (uint64_t)kb * Dm * kc, r1 = (uint64_t)Dm * kc, r2 = kc;

    const int nslices = Dm * Da * (Db / Eb);
    int sdone = 0;
    for (int g = 0; g < Dm; ++g) {
      for (int f = 0; f < Da; ++f) {
        for (int e0 = 0; e0 < Db; e0 += Eb) {  // first b1' of the slice
            const uint64_t offA = f * lst[1] + g * lst[7] + e0 * lst[3];
            const uint64_t offB = g * lst[6];
            const uint64_t uboff = (uint64_t)e0 * Db * kb;  // rows (b1' = e0, b2') of Ub
            // parity of the indices the slice fixes (alpha, a1', and b1' when Eb = 1)
            const uint32_t zs =
                z2 ? (uint32_t)(cp.par[mu][g] ^ cp.par[tv[0]][f] ^ (Eb == 1 ? cp.par[tv[1]][e0] : 0)) : 0u;
            // ---- recompute the forward intermediates and the operands, transposed ([K][rows])
            {
                XP x;  // P1
                x.tdim(Dm, lst[6], y1s[1]);
                x.tdim(Eb, lst[3], y1s[2]);
                x.tdim(Dc, lst[5], y1s[3]);
                x.tdim(Dc, lst[4], y1s[5]);
                x.tdim(Db, lst[2], y1s[6]);
                x.loops(ka, 1, y1s[0], Da, ka, y1s[4]);
                x.sum(Da, lst[0], (uint64_t)Da * ka);
                if (!x.fits(tsize - offA, usz[0], c->cap)) return set_err(HOTRG_EINVAL, "bw P1 out of bounds");
                launch_iso_expand(x.done(), T + offA, Ua, Y1, nullptr, nullptr, c->stream);
            }
            {
                XP x;  // P2
                x.tdim(ka, y1s[0], y2s[0]);
                x.tdim(Dm, y1s[1], y2s[2]);
                x.tdim(Eb, y1s[2], y2s[3]);
                x.tdim(Dc, y1s[3], y2s[4]);
                x.tdim(Da, y1s[4], y2s[5]);
                x.tdim(Dc, y1s[5], y2s[7]);
                x.loops(kb, 1, y2s[1], Db, kb, y2s[6]);
                x.sum(Db, y1s[6], (uint64_t)Db * kb);
                if (!x.fits(c->cap, usz[1], c->cap)) return set_err(HOTRG_EINVAL, "bw P2 out of bounds");
                launch_iso_expand(x.done(), Y1, Ub, Y2, nullptr, nullptr, c->stream);
            }
            {
                XP x;  // P3 -> A^T [K][M] (row length ldM); the GEMM-row dims innermost, so that
                       // neighbouring lanes write neighbouring columns of A^T
                if (z2) {  // tile layout: column-outer (a), K rows (b1', c1', a2, b2 | c2), column-inner (b, mu1 | c)
                    x.tdim(ka, y2s[0], r0);
                    x.tdim(Eb, y2s[3], ks0 * ldM);
                    x.tdim(Dc, y2s[4], ks1 * ldM);
                    x.tdim(Da, y2s[5], ks2 * ldM);
                    x.tdim(Db, y2s[6], ks3 * ldM);
                    x.tdim(kb, y2s[1], r1);
                    x.tdim(Dm, y2s[2], r2);
                    x.loops(Dc, kc, ldM, kc, 1, 1);
                } else {
                    x.tdim(Eb, y2s[3], ks0 * ldM);
                    x.tdim(Dc, y2s[4], ks1 * ldM);
                    x.tdim(Da, y2s[5], ks2 * ldM);
                    x.tdim(Db, y2s[6], ks3 * ldM);
                    x.tdim(ka, y2s[0], r0);
                    x.tdim(kb, y2s[1], r1);
                    x.tdim(Dm, y2s[2], r2);
                    x.loops(kc, 1, 1, Dc, kc, ldM);
                }
                x.sum(Dc, y2s[7], (uint64_t)Dc * kc);
                if (!x.fits(c->cap, usz[2], ldM * Ks)) return set_err(HOTRG_EINVAL, "bw P3 out of bounds");
                if (z2) {
                    // labels: summed c1, first loop c2 (old c), second loop c (new c)
                    const std::vector<uint8_t> labs[3] = {cp.par[tv[2]], cp.par[tv[2]], cp.npar[2]};
                    TRY(z2t_scatter(c, x, Uc, M, Ks, zs, zN, zKc, zld, mixed, zAT, zATh, zATl, c->ktab, 2, 1, 4,
                                    labs));
                    launch_iso_expand(x.done(), Y2, Uc, nullptr, nullptr, nullptr, c->stream);
                } else if (mixed) {
                    x.packed(ldM);
                    launch_iso_expand(x.done(), Y2, Uc, nullptr, ATh, ATl, c->stream);
                } else {
                    launch_iso_expand(x.done(), Y2, Uc, AT, nullptr, nullptr, c->stream);
                }
            }
            {
                XP x;  // Q1
                x.tdim(Dm, lst[7], z1s[1]);
                x.tdim(Da, lst[0], z1s[2]);
                x.tdim(Db, lst[2], z1s[3]);
                x.tdim(Dc, lst[4], z1s[4]);
                x.tdim(Dc, lst[5], z1s[5]);
                x.tdim(Db, lst[3], z1s[6]);
                x.loops(ka, 1, z1s[0], 1, 0, 0);
                x.sum(Da, lst[1], ka);
                if (!x.fits(tsize - offB, usz[0] - (uint64_t)f * Da * ka, c->cap))
                    return set_err(HOTRG_EINVAL, "bw Q1 out of bounds");
                launch_iso_expand(x.done(), T + offB, Ua + (size_t)f * Da * ka, Z1, nullptr, nullptr, c->stream);
            }
            {
                XP x;  // Q2
                x.tdim(ka, z1s[0], z2s[0]);
                x.tdim(Dm, z1s[1], z2s[2]);
                x.tdim(Da, z1s[2], z2s[4]);
                x.tdim(Db, z1s[3], z2s[5]);
                x.tdim(Dc, z1s[4], z2s[6]);
                x.tdim(Dc, z1s[5], z2s[7]);
                x.loops(kb, 1, z2s[1], Eb, (uint64_t)Db * kb, z2s[3]);
                x.sum(Db, z1s[6], kb);
                if (!x.fits(c->cap, usz[1] - uboff, c->cap)) return set_err(HOTRG_EINVAL, "bw Q2 out of bounds");
                launch_iso_expand(x.done(), Z1, Ub + uboff, Z2, nullptr, nullptr, c->stream);
            }
            {
                XP x;  // Q3 -> B^T [K][N] (row length ldM); GEMM-row dims innermost as in P3
                if (z2) {
                    // K in the order (b1', a2, b2, c2, c1') of ktabq, so that the
                    // product's c1' loop steps one K row; tile layout: column-outer
                    // (a'), K rows (b1', a2, b2, c2 | c1'), column-inner (b', mu2' | c')
                    const uint64_t q3 = Dc, q2 = (uint64_t)Dc * Dc, q1 = q2 * Db, q0 = q1 * Da;
                    x.tdim(ka, z2s[0], r0);
                    x.tdim(Eb, z2s[3], q0 * ldM);
                    x.tdim(Da, z2s[4], q1 * ldM);
                    x.tdim(Db, z2s[5], q2 * ldM);
                    x.tdim(Dc, z2s[6], q3 * ldM);
                    x.tdim(kb, z2s[1], r1);
                    x.tdim(Dm, z2s[2], r2);
                    x.loops(Dc, (uint64_t)Dc * kc, ldM, kc, 1, 1);
                } else {
                    x.tdim(Eb, z2s[3], ks0 * ldM);
                    x.tdim(Da, z2s[4], ks2 * ldM);
                    x.tdim(Db, z2s[5], ks3 * ldM);
                    x.tdim(Dc, z2s[6], ldM);
                    x.tdim(ka, z2s[0], r0);
                    x.tdim(kb, z2s[1], r1);
                    x.tdim(Dm, z2s[2], r2);
                    x.loops(kc, 1, 1, Dc, (uint64_t)Dc * kc, ks1 * ldM);
                }
                x.sum(Dc, z2s[7], kc);
                if (!x.fits(c->cap, usz[2], ldM * Ks)) return set_err(HOTRG_EINVAL, "bw Q3 out of bounds");
                if (z2) {
                    // labels: summed c2', first loop c1' (old c), second loop c' (new c)
                    const std::vector<uint8_t> labs[3] = {cp.par[tv[2]], cp.par[tv[2]], cp.npar[2]};
                    TRY(z2t_scatter(c, x, Uc, M, Ks, zs, zN, zKc, zld, mixed, zBT, zBTh, zBTl, c->ktabq, 3, 1, 4,
                                    labs));
                    launch_iso_expand(x.done(), Z2, Uc, nullptr, nullptr, nullptr, c->stream);
                } else if (mixed) {
                    x.packed(ldM);
                    launch_iso_expand(x.done(), Z2, Uc, nullptr, BTh, BTl, c->stream);
                } else {
                    launch_iso_expand(x.done(), Z2, Uc, BT, nullptr, nullptr, c->stream);
                }
            }
            // ---- A_bar = C_bar B, B_bar = C_bar^T A (FP64, or bf16x3 in mixed precision)
            if (z2) {
                // per inner K class b (GEMM class g = b ^ zs): A_bar_b = C_bar_g B_b,
                // B_bar_b = C_bar_g^T A_b, outputs N_g x K_b; then the natural layout
                const uint64_t sq0 = (uint64_t)zN[0] * zN[0];
                X3Gemm ga[2], gb[2];
                int n = 0;
                for (int b = 0; b < 2; ++b) {
                    const int g = b ^ (int)zs;
                    if (zN[g] == 0 || zKc[b] == 0) continue;
                    if (mixed) {
                        ga[n] = X3Gemm{zCh[g], zCl[g], zBTh[b], zBTl[b], zAo[b], (int)zN[g], 1, (int)zKc[b],
                                       (int)zld[g], zKc[b], 0};
                        gb[n] = X3Gemm{zCTh[g], zCTl[g], zATh[b], zATl[b], zBo[b], (int)zN[g], 1, (int)zKc[b],
                                       (int)zld[g], zKc[b], 0};
                        ++n;
                    } else {
                        launch_gemm_f64(Cbar + (g ? sq0 : 0), zBT[b], zAo[b], (int)zN[g], (int)zKc[b], (int)zN[g],
                                        zN[g], zld[g], zKc[b], 0, c->stream);
                        launch_gemm_f64(CbarT + (g ? sq0 : 0), zAT[b], zBo[b], (int)zN[g], (int)zKc[b], (int)zN[g],
                                        zN[g], zld[g], zKc[b], 0, c->stream);
                    }
                }
                if (mixed && n > 0) {
                    launch_gemm_bf16x3_multi(ga, n, c->stream, tail);
                    launch_gemm_bf16x3_multi(gb, n, c->stream, tail);
                }
                // (A_bar and B_bar stay in class blocks: the fused last-product
                // adjoints read them through the tables, and the natural layout
                // is written only for the generic fallback below)
            } else if (mixed) {
                launch_gemm_bf16x3(Ch, Cl, BTh, BTl, Abar, (int)M, 1, (int)Ks, (int)ldM, Ks, 0, c->stream, tail);
                launch_gemm_bf16x3(CTh, CTl, ATh, ATl, Bbar, (int)M, 1, (int)Ks, (int)ldM, Ks, 0, c->stream, tail);
            } else {
                launch_gemm_f64(Cbar, BT, Abar, (int)M, (int)Ks, (int)M, M, M, Ks, 0, c->stream);
                launch_gemm_f64(CbarT, AT, Bbar, (int)M, (int)Ks, (int)M, M, M, Ks, 0, c->stream);
            }
            TRY(check_launch(c, "reverse GEMMs"));

            // ---- A side: through P3, P2, P1
            bool fusedA = false;
            {   // Yb2 and Uc_bar (A) in one pass over A_bar (rows (a,b,mu1 | c), columns (K' | c2))
                LastProdParams lp{};
                lp.n_o1 = (uint32_t)((uint64_t)ka * kb * Dm);
                lp.n_o2 = 1;
                lp.NJ = (uint32_t)((uint64_t)Eb * Dc * Da * Db);
                lp.x_o1 = (uint32_t)(kc * Ks);
                lp.xj = Dc;
                lp.xc = (uint32_t)Ks;
                lp.xs = 1;
                lp.out_o1 = (uint32_t)y2s[2];
                lp.oj = (uint32_t)y2s[6];
                lp.ol = (uint32_t)y2s[7];
                lp.ul = (uint32_t)((uint64_t)Dc * kc);
                lp.us = (uint32_t)kc;
                lp.uc = 1;
                lp.L = kc;
                lp.N = Dc;
                if (z2) {  // A_bar's columns follow the rows of B^T (the ktabq order, listed densely by kmapq)
                    lp.cls = 1;
                    lp.blk[0] = zAo[0];
                    lp.blk[1] = zAo[1];
                    lp.ldb[0] = zKc[0];
                    lp.ldb[1] = zKc[1];
                    lp.rtab = c->rtab;
                    lp.ktab = c->kmapq;
                    lp.zs = zs;
                    lp.ks = make_fastdiv((uint32_t)Ks);
                }
                TRY(run_lastprod(c, lp, Abar, M * Ks, Y2, Uc, usz[2], Yb2, c->cap, Ubar[2], &fusedA));
            }
            if (!fusedA && z2)
                launch_z2_unscatter(zAo[0], zAo[1], zKc[0], zKc[1], c->rtab, c->kmapq, zs, 0u, (uint32_t)Ks,
                                    (uint32_t)M, Abar, c->stream);
            if (!fusedA) {   // Yb2[a,b,mu1,b1',c1',a2,b2,c1] = sum_{c,c2} Uc[(c1,c2),c] A_bar[(a,b,mu1,c),(b1',c1',a2,b2,c2)]
                EP e;
                e.o(ka, r0 * Ks, 0, y2s[0]);
                e.o(kb, r1 * Ks, 0, y2s[1]);
                e.o(Dm, r2 * Ks, 0, y2s[2]);
                e.o(Eb, ks0, 0, y2s[3]);
                e.o(Dc, ks1, 0, y2s[4]);
                e.o(Da, ks2, 0, y2s[5]);
                e.o(Db, ks3, 0, y2s[6]);
                e.o(Dc, 0, (uint64_t)Dc * kc, y2s[7]);
                e.s(kc, Ks, 1);
                e.s(Dc, 1, kc);
                TRY(run_einsum(c, e, Abar, M * Ks, Uc, usz[2], Yb2, c->cap, 1.0, 0, "bw Y2bar"));
            }
            if (!fusedA) {   // Uc_bar[(c1,c2),c] += sum Y2[.., c1] A_bar[(.., c), (.., c2)]
                EP e;
                e.o(Dc, y2s[7], 0, (uint64_t)Dc * kc);
                e.o(Dc, 0, 1, kc);
                e.o(kc, 0, Ks, 1);
                e.s(ka, y2s[0], r0 * Ks);
                e.s(kb, y2s[1], r1 * Ks);
                e.s(Dm, y2s[2], r2 * Ks);
                e.s(Eb, y2s[3], ks0);
                e.s(Dc, y2s[4], ks1);
                e.s(Da, y2s[5], ks2);
                e.s(Db, y2s[6], ks3);
                TRY(run_einsum(c, e, Y2, c->cap, Abar, M * Ks, Ubar[2], usz[2], 1.0, 1, "bw Uc_bar (A)"));
            }
            {   // Yb1[a,mu1,b1',c1',a2,c1,b1] = sum_{b,b2} Ub[(b1,b2),b] Yb2[a,b,mu1,b1',c1',a2,b2,c1]
                EP e;
                e.o(ka, y2s[0], 0, y1s[0]);
                e.o(Dm, y2s[2], 0, y1s[1]);
                e.o(Eb, y2s[3], 0, y1s[2]);
                e.o(Dc, y2s[4], 0, y1s[3]);
                e.o(Da, y2s[5], 0, y1s[4]);
                e.o(Dc, y2s[7], 0, y1s[5]);
                e.o(Db, 0, (uint64_t)Db * kb, y1s[6]);
                e.s(kb, y2s[1], 1);
                e.s(Db, y2s[6], kb);
                TRY(run_einsum(c, e, Yb2, c->cap, Ub, usz[1], Yb1, c->cap, 1.0, 0, "bw Y1bar"));
            }
            {   // Ub_bar[(b1,b2),b] += sum Y1[.., b1] Yb2[.., b, .., b2, ..]
                EP e;
                e.o(Db, y1s[6], 0, (uint64_t)Db * kb);
                e.o(Db, 0, y2s[6], kb);
                e.o(kb, 0, y2s[1], 1);
                e.s(ka, y1s[0], y2s[0]);
                e.s(Dm, y1s[1], y2s[2]);
                e.s(Eb, y1s[2], y2s[3]);
                e.s(Dc, y1s[3], y2s[4]);
                e.s(Da, y1s[4], y2s[5]);
                e.s(Dc, y1s[5], y2s[7]);
                TRY(run_einsum(c, e, Y1, c->cap, Yb2, c->cap, Ubar[1], usz[1], 1.0, 1, "bw Ub_bar (A)"));
            }
            {   // Tprev[a1,f,b1,b1',c1,c1',mu1,g] += sum_{a,a2} Ua[(a1,a2),a] Yb1[a,mu1,b1',c1',a2,c1,b1]
                EP e;
                e.o(Da, 0, (uint64_t)Da * ka, lst[0]);
                e.o(Db, y1s[6], 0, lst[2]);
                e.o(Eb, y1s[2], 0, lst[3]);
                e.o(Dc, y1s[5], 0, lst[4]);
                e.o(Dc, y1s[3], 0, lst[5]);
                e.o(Dm, y1s[1], 0, lst[6]);
                e.s(ka, y1s[0], 1);
                e.s(Da, y1s[4], ka);
                TRY(run_einsum(c, e, Yb1, c->cap, Ua, usz[0], Tprev + offA, tsize - offA, 1.0, 1, "bw T1bar"));
            }
            {   // Ua_bar[(a1,a2),a] += sum T[a1,f,..,g] Yb1[a,..,a2,..]
                EP e;
                e.o(Da, lst[0], 0, (uint64_t)Da * ka);
                e.o(Da, 0, y1s[4], ka);
                e.o(ka, 0, y1s[0], 1);
                e.s(Dm, lst[6], y1s[1]);
                e.s(Eb, lst[3], y1s[2]);
                e.s(Dc, lst[5], y1s[3]);
                e.s(Dc, lst[4], y1s[5]);
                e.s(Db, lst[2], y1s[6]);
                TRY(run_einsum(c, e, T + offA, tsize - offA, Yb1, c->cap, Ubar[0], usz[0], 1.0, 1, "bw Ua_bar (A)"));
            }
            // ---- B side: through Q3, Q2, Q1
            bool fusedB = false;
            {   // Zb2 and Uc_bar (B) in one pass over B_bar (rows (a',b',mu2' | c'), columns
                // (b1' | c1' | a2,b2,c2))
                LastProdParams lp{};
                lp.n_o1 = (uint32_t)((uint64_t)ka * kb * Dm);
                lp.n_o2 = (uint32_t)Eb;
                lp.NJ = (uint32_t)((uint64_t)Da * Db * Dc);
                lp.x_o1 = (uint32_t)(kc * Ks);
                lp.x_o2 = (uint32_t)ks0;
                lp.xj = 1;
                lp.xc = (uint32_t)Ks;
                lp.xs = (uint32_t)ks1;
                lp.out_o1 = (uint32_t)z2s[2];
                lp.out_o2 = (uint32_t)z2s[3];
                lp.oj = (uint32_t)z2s[6];
                lp.ol = (uint32_t)z2s[7];
                lp.ul = (uint32_t)kc;
                lp.us = (uint32_t)((uint64_t)Dc * kc);
                lp.uc = 1;
                lp.L = kc;
                lp.N = Dc;
                if (z2) {  // B_bar's columns follow the rows of A^T (the dense order of ktab)
                    lp.cls = 1;
                    lp.blk[0] = zBo[0];
                    lp.blk[1] = zBo[1];
                    lp.ldb[0] = zKc[0];
                    lp.ldb[1] = zKc[1];
                    lp.rtab = c->rtab;
                    lp.ktab = c->ktab;
                    lp.zs = zs;
                    lp.ks = make_fastdiv((uint32_t)Ks);
                }
                TRY(run_lastprod(c, lp, Bbar, M * Ks, Z2, Uc, usz[2], Yb2, c->cap, Ubar[2], &fusedB));
            }
            if (!fusedB && z2)
                launch_z2_unscatter(zBo[0], zBo[1], zKc[0], zKc[1], c->rtab, c->ktab, zs, 0u, (uint32_t)Ks,
                                    (uint32_t)M, Bbar, c->stream);
            if (!fusedB) {   // Zb2[a',b',mu2',b1',a2,b2,c2,c2'] = sum_{c',c1'} Uc[(c1',c2'),c'] B_bar[(a',b',mu2',c'),(b1',c1',a2,b2,c2)]
                EP e;
                e.o(ka, r0 * Ks, 0, z2s[0]);
                e.o(kb, r1 * Ks, 0, z2s[1]);
                e.o(Dm, r2 * Ks, 0, z2s[2]);
                e.o(Eb, ks0, 0, z2s[3]);
                e.o(Da, ks2, 0, z2s[4]);
                e.o(Db, ks3, 0, z2s[5]);
                e.o(Dc, 1, 0, z2s[6]);
                e.o(Dc, 0, kc, z2s[7]);
                e.s(kc, Ks, 1);
                e.s(Dc, ks1, (uint64_t)Dc * kc);
                TRY(run_einsum(c, e, Bbar, M * Ks, Uc, usz[2], Yb2, c->cap, 1.0, 0, "bw Z2bar"));
            }
            if (!fusedB) {   // Uc_bar[(c1',c2'),c'] += sum Z2[.., c2'] B_bar[(.., c'), (b1', c1', ..)]
                EP e;
                e.o(Dc, 0, ks1, (uint64_t)Dc * kc);
                e.o(Dc, z2s[7], 0, kc);
                e.o(kc, 0, Ks, 1);
                e.s(ka, z2s[0], r0 * Ks);
                e.s(kb, z2s[1], r1 * Ks);
                e.s(Dm, z2s[2], r2 * Ks);
                e.s(Eb, z2s[3], ks0);
                e.s(Da, z2s[4], ks2);
                e.s(Db, z2s[5], ks3);
                e.s(Dc, z2s[6], 1);
                TRY(run_einsum(c, e, Z2, c->cap, Bbar, M * Ks, Ubar[2], usz[2], 1.0, 1, "bw Uc_bar (B)"));
            }
            {   // Zb1[a',mu2',a2,b2,c2,c2',b2'] = sum_{b',b1'} Ub[(b1',b2'),b'] Zb2[a',b',mu2',b1',a2,b2,c2,c2']
                EP e;
                e.o(ka, z2s[0], 0, z1s[0]);
                e.o(Dm, z2s[2], 0, z1s[1]);
                e.o(Da, z2s[4], 0, z1s[2]);
                e.o(Db, z2s[5], 0, z1s[3]);
                e.o(Dc, z2s[6], 0, z1s[4]);
                e.o(Dc, z2s[7], 0, z1s[5]);
                e.o(Db, 0, kb, z1s[6]);
                e.s(kb, z2s[1], 1);
                e.s(Eb, z2s[3], (uint64_t)Db * kb);
                TRY(run_einsum(c, e, Yb2, c->cap, Ub + uboff, usz[1] - uboff, Yb1, c->cap, 1.0, 0, "bw Z1bar"));
            }
            {   // Ub_bar[(b1',b2'),b'] += sum Z1[.., b2'] Zb2[.., b', .., b1', ..]
                EP e;
                e.o(Eb, 0, z2s[3], (uint64_t)Db * kb);
                e.o(Db, z1s[6], 0, kb);
                e.o(kb, 0, z2s[1], 1);
                e.s(ka, z1s[0], z2s[0]);
                e.s(Dm, z1s[1], z2s[2]);
                e.s(Da, z1s[2], z2s[4]);
                e.s(Db, z1s[3], z2s[5]);
                e.s(Dc, z1s[4], z2s[6]);
                e.s(Dc, z1s[5], z2s[7]);
                TRY(run_einsum(c, e, Z1, c->cap, Yb2, c->cap, Ubar[1] + uboff, usz[1] - uboff, 1.0, 1,
                               "bw Ub_bar (B)"));
            }
            {   // Tprev[a2,a2',b2,b2',c2,c2',g,mu2'] += sum_{a'} Ua[(f,a2'),a'] Zb1[a',mu2',a2,b2,c2,c2',b2']
                EP e;
                e.o(Da, z1s[2], 0, lst[0]);
                e.o(Da, 0, ka, lst[1]);
                e.o(Db, z1s[3], 0, lst[2]);
                e.o(Db, z1s[6], 0, lst[3]);
                e.o(Dc, z1s[4], 0, lst[4]);
                e.o(Dc, z1s[5], 0, lst[5]);
                e.o(Dm, z1s[1], 0, lst[7]);
                e.s(ka, z1s[0], 1);
                TRY(run_einsum(c, e, Yb1, c->cap, Ua + (size_t)f * Da * ka, usz[0] - (uint64_t)f * Da * ka,
                               Tprev + offB, tsize - offB, 1.0, 1, "bw T2bar"));
            }
            {   // Ua_bar[(f,a2'),a'] += sum T[a2,a2',..,g,mu2'] Zb1[a',mu2',a2,..]
                EP e;
                e.o(Da, lst[1], 0, ka);
                e.o(ka, 0, z1s[0], 1);
                e.s(Da, lst[0], z1s[2]);
                e.s(Db, lst[2], z1s[3]);
                e.s(Db, lst[3], z1s[6]);
                e.s(Dc, lst[4], z1s[4]);
                e.s(Dc, lst[5], z1s[5]);
                e.s(Dm, lst[7], z1s[1]);
                TRY(run_einsum(c, e, T + offB, tsize - offB, Yb1, c->cap, Ubar[0] + (size_t)f * Da * ka,
                               usz[0] - (uint64_t)f * Da * ka, 1.0, 1, "bw Ua_bar (B)"));
            }
            TRY(report_progress(c, "reverse", step, ++sdone, nslices));
        }
      }
    }

    // ---- isometries -> environments -> T (truncated axes only)
    for (int i = 0; i < 3; ++i) {
        if (!cp.trunc[i]) continue;
        const int Dn = ldim[2 * i], n = cp.n[i], k = cp.k[i];
        double *Ebar = c->E;  // scratch: n x n
        launch_eigh_adjoint(cp.V[i], cp.lam[i], Ubar[i], n, k, Ebar, c->stream);
        TRY(check_launch(c, "eigh adjoint"));
        const int leg = 2 * i + cp.side[i];
        double *G1 = c->G, *G2 = c->G + (size_t)kMaxEnvN * kMaxEnvN;
        double *G1b = c->E + (size_t)2 * kMaxEnvN * kMaxEnvN, *G2b = c->E + (size_t)3 * kMaxEnvN * kMaxEnvN;
        TRY(gram(c, T, lst, ldim, leg, 7, G1));
        TRY(gram(c, T, lst, ldim, leg, 6, G2));
        const uint64_t R = (uint64_t)Dn * Dm, RR = R * R, nn = (uint64_t)n * n;
        {   // G1bar[(p,a),(p',a')] = sum_{q,q'} Ebar[(p,q),(p',q')] G2[(q,a),(q',a')]
            EP e;
            e.o(Dn, (uint64_t)Dn * n, 0, Dm * R);
            e.o(Dm, 0, R, R);
            e.o(Dn, Dn, 0, Dm);
            e.o(Dm, 0, 1, 1);
            e.s(Dn, n, Dm * R);
            e.s(Dn, 1, Dm);
            TRY(run_einsum(c, e, Ebar, nn, G2, RR, G1b, RR, 1.0, 0, "bw G1bar"));
        }
        {   // G2bar[(q,a),(q',a')] = sum_{p,p'} Ebar[(p,q),(p',q')] G1[(p,a),(p',a')]
            EP e;
            e.o(Dn, n, 0, Dm * R);
            e.o(Dm, 0, R, R);
            e.o(Dn, 1, 0, Dm);
            e.o(Dm, 0, 1, 1);
            e.s(Dn, (uint64_t)Dn * n, Dm * R);
            e.s(Dn, Dn, Dm);
            TRY(run_einsum(c, e, Ebar, nn, G1, RR, G2b, RR, 1.0, 0, "bw G2bar"));
        }
        // X_bar = (G_bar + G_bar^T) X for each Gram, scattered back into Tprev
        for (int gsel = 0; gsel < 2; ++gsel) {
            const double *Gb = gsel == 0 ? G1b : G2b;
            const int la = gsel == 0 ? 7 : 6;
            for (int tr = 0; tr < 2; ++tr) {
                EP e;
                const uint64_t sp = tr ? Dm : Dm * R, sa = tr ? 1 : R;       // strides of (p, a) in G_bar
                const uint64_t sp2 = tr ? Dm * R : Dm, sa2 = tr ? R : 1;     // strides of (p', a')
                for (int l = 0; l < 8; ++l) {
                    if (l == leg) e.o(Dn, sp, 0, lst[l]);
                    else if (l == la) e.o(Dm, sa, 0, lst[l]);
                    else e.o(ldim[l], 0, lst[l], lst[l]);
                }
                e.s(Dn, sp2, lst[leg]);
                e.s(Dm, sa2, lst[la]);
                TRY(run_einsum(c, e, Gb, RR, T, tsize, Tprev, tsize, 1.0, 1, "bw Gram"));
            }
        }
    }
    return HOTRG_OK;
}

int backward(hotrg_ctx *c, double *dbeta, double *dh) {
    if (c->failed) return set_err(HOTRG_ESTATE, "context is in a failed state");
    if (!c->cfg.keep_checkpoints) return set_err(HOTRG_ESTATE, "hotrg_backward needs keep_checkpoints = 1");
    if (c->ckpt_broken || (int)c->ckpts.size() != c->n)
        return set_err(HOTRG_ESTATE, "checkpoints do not cover the flow from the initial tensor");
    if (!(c->beta > 1e-3)) return set_err(HOTRG_EINVAL, "hotrg_backward needs beta > 1e-3");
    // a cut inside a degenerate multiplet has no eigenvector derivative
    // (1 / (lam_i - lam_j) with lam_i = lam_j); refused before any device work
    for (size_t s = 0; s < c->ckpts.size(); ++s)
        for (int i = 0; i < 3; ++i)
            if (c->ckpts[s].flagged[i])
                return set_err(HOTRG_ENUMERIC, "step " + std::to_string(s + 1) + ", axis " +
                                                   std::to_string(c->ckpts[s].tv[i]) +
                                                   ": the cut has no spectral gap above tau, the derivative of "
                                                   "the isometry is undefined");
    double tr, trm, tre;
    TRY(read_obs(c, &tr, &trm, &tre, nullptr));
    if (!(tr > 0) || !std::isfinite(tr)) {
        c->failed = true;
        return set_err(HOTRG_ENUMERIC, "Tr T is not finite and positive");
    }
    double *Tb, *Tp;
    TRY(bw_buf(c, BW_TBAR0, c->cap, &Tb));
    TRY(bw_buf(c, BW_TBAR1, c->cap, &Tp));
    // seed: d(lnZ/N)/dT^(n) = 2^-n delta_diag / Tr T^(n)
    uint64_t cst[8];
    canon_strides(c->dims, cst);
    uint32_t dst[4];
    for (int q = 0; q < 4; ++q) dst[q] = (uint32_t)(cst[2 * q] + cst[2 * q + 1]);
    launch_zero(Tb, tensor_size(c->dims), c->stream);
    launch_diag_set(Tb, c->dims, dst, std::ldexp(1.0 / tr, -c->n), c->stream);
    for (int k = c->n - 1; k >= 0; --k) {
        // the precision of step k + 1 in the forward flow
        const bool mixed = c->cfg.precision == HOTRG_BF16X3 && (k + 1) >= c->cfg.mixed_from_step;
        TRY(backward_step(c, c->ckpts[k], Tb, Tp, mixed, k + 1));
        std::swap(Tb, Tp);
    }
    // d T^(0) / d(beta, h): W[0] = (sqrt cosh b, sqrt sinh b), V = e^{+-b h}
    const double b = c->beta, h = c->h;
    const double wc = std::sqrt(std::cosh(b)), ws = std::sqrt(std::sinh(b));
    const double dwc = std::sinh(b) / (2 * wc), dws = std::cosh(b) / (2 * ws);
    launch_site_dot(Tb, wc, ws, dwc, dws, b, h, std::exp(b * h), std::exp(-b * h), 1.0 / c->c0, c->scal,
                    c->stream);
    TRY(check_launch(c, "site derivative"));
    double out[2];
    HIP_TRY(c, hipMemcpyAsync(out, c->scal, sizeof(out), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!std::isfinite(out[0]) || !std::isfinite(out[1])) {
        c->failed = true;
        return set_err(HOTRG_ENUMERIC, "reverse pass produced a non-finite derivative");
    }
    *dbeta = out[0];
    *dh = out[1];
    return HOTRG_OK;
}

}  // namespace

// Observables from the traces of Eq. (2.5) and the A matrix of Eq. (3.2)
// (Da x Da): ln Z / N, the impurity ratios of Eqs. (2.10), (2.12), and X of
// Eq. (3.3).  Shared by hotrg_observables and hotrg_observables_noalloc.
void obs_from_traces(double tr, double trm, double tre, const double *A, int Da, int n, double lnz_acc, double h,
                     bool imp, hotrg_obs *o) {
    // a state set by the caller may have Tr <= 0; ln Z is then undefined (NaN)
    o->lnz_per_site = (tr > 0 && std::isfinite(tr)) ? lnz_acc + std::ldexp(std::log(tr), -n) : NAN;
    o->trace = tr;
    if (imp) {
        o->m_imp = trm / tr;
        o->nn_imp = tre / tr;
        o->e_imp = -4.0 * o->nn_imp - h * o->m_imp;
    } else {
        o->m_imp = o->nn_imp = o->e_imp = NAN;
    }
    double trA = 0, trA2 = 0;
    for (int t = 0; t < Da; ++t) {
        trA += A[(size_t)t * Da + t];
        for (int u = 0; u < Da; ++u) trA2 += A[(size_t)t * Da + u] * A[(size_t)u * Da + t];
    }
    o->X = trA * trA / trA2;
}

// ---- scratch of the no-allocation entry point ------------------------------
// Device memory for the trace kernel's partial results (the three traces and
// the A matrix) when the caller cannot allocate: one file-scope array per
// GPU, alive until the process ends.  Host code never uses the array's name
// as an address: the device address comes from hipGetSymbolAddress, once per
// device (with that device current), and is kept in g_scratch_ptr.
constexpr int kNoallocMaxDim = 13;
constexpr int kScratchDoubles = 3 + kNoallocMaxDim * kNoallocMaxDim;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_err(HOTRG_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_err(HOTRG_EDEVICE, "device id out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_err(HOTRG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return HOTRG_OK;
}

// =============================================================== C ABI ====
extern "C" {

int hotrg_observables_noalloc(const double *T, const double *Sm, const double *Se, const int dims[4], int axis,
                              double h, int n, double lnz_acc, void *stream, hotrg_obs *out) {
    if (!T || !dims || !out) return set_err(HOTRG_EINVAL, "null argument");
    if (axis < 0 || axis > 3) return set_err(HOTRG_EINVAL, "axis must be 0..3");
    if (n < 0 || !std::isfinite(h) || !std::isfinite(lnz_acc)) return set_err(HOTRG_EINVAL, "bad n, h or lnz_acc");
    if ((Sm == nullptr) != (Se == nullptr)) return set_err(HOTRG_EINVAL, "give both impure tensors or neither");
    for (int q = 0; q < 4; ++q)
        if (dims[q] < 1 || dims[q] > kNoallocMaxDim)
            return set_err(HOTRG_EINVAL, "hotrg_observables_noalloc: bond dimensions must be in 1.." +
                                             std::to_string(kNoallocMaxDim) + " (scratch holds " +
                                             std::to_string(kScratchDoubles) + " doubles)");
    double *sp = nullptr;
    TRY(scratch_for_current_device(&sp));
    hipStream_t st = (hipStream_t)stream;
    launch_trace_obs(T, Sm, Se, dims, axis, sp, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(HOTRG_EDEVICE, std::string("trace kernel: ") + hipGetErrorString(e));
    const int Da = dims[axis];
    double hbuf[kScratchDoubles];
    e = hipMemcpyAsync(hbuf, sp, sizeof(double) * (3 + (size_t)Da * Da), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_err(HOTRG_EDEVICE, std::string("scratch copy: ") + hipGetErrorString(e));
    std::memset(out, 0, sizeof(*out));
    out->n = n;
    for (int q = 0; q < 4; ++q) {
        out->dims[q] = dims[q];
        out->last_side[q] = -1;
    }
    obs_from_traces(hbuf[0], hbuf[1], hbuf[2], hbuf + 3, Da, n, lnz_acc, h, Sm != nullptr, out);
    out->last_axis = axis;
    out->min_cut_gap = INFINITY;
    return HOTRG_OK;
}

const char *hotrg_last_error(void) { return g_err.c_str(); }

int hotrg_init_ex(double beta, double h, int dcut, const hotrg_config *cfg, hotrg_ctx **out) {
    if (!out) return set_err(HOTRG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!(beta >= 0) || !std::isfinite(beta)) return set_err(HOTRG_EINVAL, "beta must be finite and >= 0");
    if (!std::isfinite(h)) return set_err(HOTRG_EINVAL, "h must be finite");
    if (dcut < 1 || dcut > 13) return set_err(HOTRG_EINVAL, "dcut must be in 1..13");
    hotrg_ctx *c = new hotrg_ctx();
    c->beta = beta;
    c->h = h;
    c->dcut = dcut;
    if (cfg) c->cfg = *cfg;
    else {
        c->cfg.impurities = 1;
    }
    if (c->cfg.precision != HOTRG_FP64 && c->cfg.precision != HOTRG_BF16X3) {
        delete c;
        return set_err(HOTRG_EINVAL, "unknown precision");
    }
    if (c->cfg.mixed_from_step <= 0) c->cfg.mixed_from_step = 4;
    if (c->cfg.eig_max_sweeps <= 0) c->cfg.eig_max_sweeps = 40;
    if (c->cfg.eig_max_sweeps > 1000) {
        delete c;
        return set_err(HOTRG_EINVAL, "eig_max_sweeps must be at most 1000");
    }
    if ((c->cfg.alloc == nullptr) != (c->cfg.free == nullptr)) {
        delete c;
        return set_err(HOTRG_EINVAL, "alloc and free must be given together");
    }
    if (!(c->cfg.tau_deg > 0)) c->cfg.tau_deg = 1e-12;
    c->stream = (hipStream_t)c->cfg.stream;
    const int Dmax = std::max(dcut, 2);
    size_t cap = 1;
    for (int i = 0; i < 8; ++i) cap *= (size_t)Dmax;
    c->cap = cap;
    const size_t E2 = (size_t)kMaxEnvN * kMaxEnvN;
    int rc = HOTRG_OK;
    auto fail = [&](int r) {
        hotrg_free(c);
        return r;
    };
    for (int t = 0; t < 3; ++t)
        if ((rc = alloc_n(c, &c->state[t], cap))) return fail(rc);
    if ((rc = alloc_n(c, &c->cbuf, 3 * cap))) return fail(rc);
    if ((rc = alloc_n(c, &c->gram_x, cap))) return fail(rc);
    if ((rc = alloc_n(c, &c->y1, cap))) return fail(rc);
    if ((rc = alloc_n(c, &c->y2, cap))) return fail(rc);
    c->gram_part_cap = (size_t)1024 * E2;
    if ((rc = alloc_n(c, &c->gram_part, c->gram_part_cap))) return fail(rc);
    if ((rc = alloc_n(c, &c->G, 2 * E2))) return fail(rc);
    if ((rc = alloc_n(c, &c->E, 6 * E2))) return fail(rc);
    if ((rc = alloc_n(c, &c->lam, 6 * (size_t)kMaxEnvN))) return fail(rc);
    if ((rc = alloc_n(c, &c->V, 6 * E2))) return fail(rc);
    if ((rc = alloc_n(c, &c->jwork, (size_t)4 * (kMaxEnvN + 1) * (kMaxEnvN + 1)))) return fail(rc);
    if ((rc = alloc_n(c, &c->sweeps, 8))) return fail(rc);
    if ((rc = alloc_n(c, &c->resid, 8))) return fail(rc);
    for (int i = 0; i < 3; ++i)
        if ((rc = alloc_n(c, &c->U[i], E2))) return fail(rc);
    if ((rc = alloc_n(c, &c->partials, 1024))) return fail(rc);
    if ((rc = alloc_n(c, &c->scal, 64))) return fail(rc);
    if ((rc = alloc_n(c, &c->obs, 3 + (size_t)kMaxEnvN))) return fail(rc);

    // T^(0), S^(0) (Eqs. (2.2), (2.6)); W from the bond matrix (Eq. (2.1))
    const double wc = std::sqrt(std::cosh(beta)), ws = std::sqrt(std::sinh(beta));
    launch_init_site(c->state[0], c->state[1], wc, ws, wc, -ws, std::exp(beta * h), std::exp(-beta * h), c->stream);
    launch_sumsq(c->state[0], 256, c->partials, 1, c->scal, c->stream);
    double ss = 0;
    if (hipMemcpyAsync(&ss, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(set_err(HOTRG_EDEVICE, "initial tensor upload failed"));
    double c0 = std::sqrt(ss);
    if (!(c0 > 0) || !std::isfinite(c0)) return fail(set_err(HOTRG_ENUMERIC, "initial norm not finite"));
    int ext[1] = {256};
    uint32_t st[1] = {1};
    PermParams pp = perm_params(1, ext, st);
    launch_permute(pp, c->state[0], c->cbuf, 1.0 / c0, c->stream);
    launch_permute(pp, c->state[1], c->cbuf + 256, 1.0 / c0, c->stream);
    launch_permute(pp, c->cbuf, c->state[0], 1.0, c->stream);
    launch_permute(pp, c->cbuf + 256, c->state[1], 1.0, c->stream);
    launch_permute(pp, c->cbuf + 256, c->state[2], 1.0, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(set_err(HOTRG_EDEVICE, "init kernels failed"));
    c->lnz_acc = std::log(c0);
    c->c0 = c0;
    // at h = 0 the bond index 0 (column (1, 1) of W) is Z2-even, index 1 odd
    c->z2 = (h == 0.0);
    for (int q = 0; q < 4; ++q) c->par[q] = {0, 1};
    *out = c;
    return HOTRG_OK;
}

int hotrg_init(double beta, double h, int dcut, hotrg_ctx **out) { return hotrg_init_ex(beta, h, dcut, nullptr, out); }

int hotrg_step(hotrg_ctx *ctx, int axis) { return do_step(ctx, axis, nullptr, nullptr); }

int hotrg_step_with_isometries(hotrg_ctx *ctx, int axis, const double *const U[4], const int k[4]) {
    if (!U || !k) return set_err(HOTRG_EINVAL, "U or k is NULL");
    return do_step(ctx, axis, U, k);
}

int hotrg_truncate(hotrg_ctx *c, int axis) {
    if (!c) return set_err(HOTRG_EINVAL, "null context");
    if (c->failed) return set_err(HOTRG_ESTATE, "context is in a failed state");
    if (axis < 0 || axis > 3) return set_err(HOTRG_EINVAL, "axis must be 0..3");
    int tv[3];
    transverse_of(axis, tv);
    uint64_t lst[8];
    int ldim[8];
    local_legs(c->dims, axis, tv, lst, ldim);
    int k[3];
    TRY(isometries(c, c->state[0], lst, ldim, tv, axis, k));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return HOTRG_OK;
}

int hotrg_lnZ(hotrg_ctx *c, double *lnz) {
    if (!c || !lnz) return set_err(HOTRG_EINVAL, "null argument");
    if (c->failed) return set_err(HOTRG_ESTATE, "context is in a failed state");
    double tr, trm, tre;
    TRY(read_obs(c, &tr, &trm, &tre, nullptr));
    if (!(tr > 0) || !std::isfinite(tr)) {
        c->failed = true;
        return set_err(HOTRG_ENUMERIC, "Tr T is not finite and positive");
    }
    *lnz = c->lnz_acc + std::ldexp(std::log(tr), -c->n);
    return HOTRG_OK;
}

int hotrg_observables(hotrg_ctx *c, hotrg_obs *o) {
    if (!c || !o) return set_err(HOTRG_EINVAL, "null argument");
    if (c->failed) return set_err(HOTRG_ESTATE, "context is in a failed state");
    double tr, trm, tre;
    std::vector<double> A;
    TRY(read_obs(c, &tr, &trm, &tre, &A));
    std::memset(o, 0, sizeof(*o));
    o->n = c->n;
    for (int q = 0; q < 4; ++q) o->dims[q] = c->dims[q];
    obs_from_traces(tr, trm, tre, A.data(), c->dims[c->last_axis < 0 ? 3 : c->last_axis], c->n, c->lnz_acc, c->h,
                    c->cfg.impurities != 0, o);
    o->last_axis = c->last_axis;
    o->min_cut_gap = c->min_gap;
    o->flagged = c->flagged;
    for (int q = 0; q < 4; ++q) {
        o->last_side[q] = c->dec[q].truncated ? c->dec[q].side : -1;
        o->last_k[q] = c->dec[q].k;
        o->last_eps[q] = c->dec[q].side == 1 ? c->dec[q].eps_f : c->dec[q].eps_b;
    }
    o->last_cn = c->last_cn;
    o->device_bytes = c->device_bytes;
    o->eig_sweeps = c->eig_sweeps;
    o->eig_residual = c->eig_resid;
    o->block_sparse = c->n > 0 && c->step_z2 ? 1 : 0;
    return HOTRG_OK;
}

int hotrg_backward(hotrg_ctx *c, double *dbeta, double *dh) {
    if (!c || !dbeta || !dh) return set_err(HOTRG_EINVAL, "null argument");
    return backward(c, dbeta, dh);
}

void hotrg_free(hotrg_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    for (auto &o : c->owned)
        if (o.p) release(c, o.p);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto e : c->ph)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

int hotrg_get_dims(hotrg_ctx *c, int dims[4], int *n) {
    if (!c || !dims) return set_err(HOTRG_EINVAL, "null argument");
    for (int q = 0; q < 4; ++q) dims[q] = c->dims[q];
    if (n) *n = c->n;
    return HOTRG_OK;
}

int hotrg_get_tensor(hotrg_ctx *c, int which, double *out, size_t count) {
    if (!c || !out) return set_err(HOTRG_EINVAL, "null argument");
    if (which < 0 || which > 2) return set_err(HOTRG_EINVAL, "which must be 0, 1 or 2");
    if (which > 0 && !c->cfg.impurities) return set_err(HOTRG_ESTATE, "impurities are off");
    size_t need = tensor_size(c->dims);
    if (count < need) return set_err(HOTRG_EINVAL, "output buffer too small");
    HIP_TRY(c, hipMemcpyAsync(out, c->state[which], sizeof(double) * need, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return HOTRG_OK;
}

int hotrg_set_state(hotrg_ctx *c, const int dims[4], const double *T, const double *Sm, const double *Se, int n,
                    double lnz_acc) {
    if (!c || !dims || !T) return set_err(HOTRG_EINVAL, "null argument");
    if (c->failed) return set_err(HOTRG_ESTATE, "context is in a failed state");
    const int Dmax = std::max(c->dcut, 2);
    for (int q = 0; q < 4; ++q)
        if (dims[q] < 1 || dims[q] > Dmax) return set_err(HOTRG_EINVAL, "dims out of range");
    if (c->cfg.impurities && (!Sm || !Se)) return set_err(HOTRG_EINVAL, "impure tensors required");
    if (n < 0) return set_err(HOTRG_EINVAL, "n must be >= 0");
    // steps before this state are unknown: the reverse pass cannot reach beta,
    // h, so the stored checkpoints are dropped (and their memory returned)
    TRY(clear_checkpoints(c));
    size_t need = tensor_size(dims);
    HIP_TRY(c, hipMemcpyAsync(c->state[0], T, sizeof(double) * need, hipMemcpyHostToDevice, c->stream));
    if (c->cfg.impurities) {
        HIP_TRY(c, hipMemcpyAsync(c->state[1], Sm, sizeof(double) * need, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->state[2], Se, sizeof(double) * need, hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int q = 0; q < 4; ++q) c->dims[q] = dims[q];
    c->n = n;
    c->lnz_acc = lnz_acc;
    c->first_axis = n > 0 ? 0 : -1;
    c->last_axis = -1;
    c->ckpt_broken = true;
    c->step_z2 = false;
    // Z2 labels for a state given by the caller: at h = 0, bond parity
    // i mod 2 if T and S_e vanish on every odd-parity entry and S_m on every
    // even one (exactly); otherwise the state carries no labels
    c->z2 = false;
    if (c->h == 0.0) {
        bool ok = true;
        const double *ts[3] = {T, c->cfg.impurities ? Sm : nullptr, c->cfg.impurities ? Se : nullptr};
        int ext[8];
        for (int l = 0; l < 8; ++l) ext[l] = dims[l / 2];
        for (int t = 0; t < 3 && ok; ++t) {
            if (!ts[t]) continue;
            const int want = t == 1 ? 1 : 0;
            int idx[8] = {0, 0, 0, 0, 0, 0, 0, 0}, par = 0;
            for (size_t e = 0; e < need; ++e) {
                if (ts[t][e] != 0.0 && par != want) {
                    ok = false;
                    break;
                }
                // next multi-index (last leg fastest), parity updated incrementally
                for (int l = 7; l >= 0; --l) {
                    par ^= idx[l] & 1;
                    if (++idx[l] < ext[l]) {
                        par ^= idx[l] & 1;
                        break;
                    }
                    idx[l] = 0;
                }
            }
        }
        if (ok) {
            c->z2 = true;
            for (int q = 0; q < 4; ++q) {
                c->par[q].resize(dims[q]);
                for (int i = 0; i < dims[q]; ++i) c->par[q][i] = (uint8_t)(i & 1);
            }
        }
    }
    return HOTRG_OK;
}

int hotrg_get_isometry(hotrg_ctx *c, int q, double *out, size_t count, int *rows, int *cols) {
    if (!c || !out || q < 0 || q > 3) return set_err(HOTRG_EINVAL, "bad argument");
    if (c->iso_axis < 0 || q == c->iso_axis) return set_err(HOTRG_ESTATE, "no isometry for this axis");
    int tv[3];
    transverse_of(c->iso_axis, tv);
    int i = (q == tv[0]) ? 0 : (q == tv[1] ? 1 : 2);
    size_t need = (size_t)c->Urows[q] * c->Ucols[q];
    if (count < need) return set_err(HOTRG_EINVAL, "output buffer too small");
    HIP_TRY(c, hipMemcpyAsync(out, c->U[i], sizeof(double) * need, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (rows) *rows = c->Urows[q];
    if (cols) *cols = c->Ucols[q];
    return HOTRG_OK;
}

int hotrg_get_spectrum(hotrg_ctx *c, int q, int side, double *out, size_t count, int *len) {
    if (!c || q < 0 || q > 3 || side < 0 || side > 1) return set_err(HOTRG_EINVAL, "bad argument");
    const auto &s = c->spectra[q][side];
    if (len) *len = (int)s.size();
    if (out) {
        if (count < s.size()) return set_err(HOTRG_EINVAL, "output buffer too small");
        std::copy(s.begin(), s.end(), out);
    }
    return HOTRG_OK;
}

int hotrg_kernel_stats(hotrg_ctx *c, int kernel, double *ms, long long *launches, double *flops) {
    if (!c || kernel < 0 || kernel > 5) return set_err(HOTRG_EINVAL, "bad argument");
    if (kernel == 0) {
        if (ms) *ms = c->gemm_ms;
        if (launches) *launches = c->gemm_launches;
        if (flops) *flops = c->gemm_flops;
        return HOTRG_OK;
    }
    if (kernel == 4 || kernel == 5) {
        if (ms) *ms = 0.0;
        if (launches) *launches = kernel == 4 ? c->z2_tile_launches : c->z2_rev_steps;
        if (flops) *flops = 0.0;
        return HOTRG_OK;
    }
    TRY(flush_phases(c));
    if (ms) *ms = c->phase_ms[kernel - 1];
    if (launches) *launches = c->phase_steps;
    if (flops) *flops = kernel == 2 ? c->gemm_flops : 0.0;
    return HOTRG_OK;
}

int hotrg_reset_stats(hotrg_ctx *c) {
    if (!c) return set_err(HOTRG_EINVAL, "null context");
    TRY(flush_phases(c));
    for (double &m : c->phase_ms) m = 0;
    c->phase_steps = 0;
    c->gemm_ms = 0;
    c->gemm_launches = 0;
    c->gemm_flops = 0;
    c->z2_tile_launches = 0;
    c->z2_rev_steps = 0;
    return HOTRG_OK;
}

}  // extern "C"
