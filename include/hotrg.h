/*
 * hotrg.h -- C ABI of the MI355X (gfx950) HOTRG library for the 4D Ising model.
 *
 * Method: Akiyama, Kuramashi, Yamashita, Yoshimura, "Phase transition of
 * four-dimensional Ising model with higher-order tensor renormalization
 * group" (arXiv:1906.06060), Sec. 2.  The library holds one coarse-graining
 * state (T, and the impure tensors S_m, S_e) in device memory and advances it
 * one direction at a time.
 *
 * Conventions shared by every call
 *   - Tensors are rank 8 with legs (x, x', y, y', z, z', t, t') in row-major
 *     order (leg x outermost, t' contiguous), FP64.  Leg q is the backward,
 *     q' the forward bond of axis q; backward and forward legs of one axis
 *     share a dimension D_q.  Axis ids: 0 = x, 1 = y, 2 = z, 3 = t.
 *   - All device work is enqueued on the stream given in hotrg_config
 *     (a hipStream_t; NULL = the default stream).  Calls that return host
 *     values synchronise that stream before returning.
 *   - Every call returns an int status (HOTRG_OK = 0 or a negative code);
 *     no C++ exception crosses the ABI.  hotrg_last_error() gives a
 *     thread-local message for the last failure on the calling thread.
 *   - Ownership: the context owns every device buffer it holds; they come
 *     from the caller's allocator when hotrg_config.alloc / free are given
 *     (a framework's caching allocator, for instance), else from hipMalloc,
 *     and hotrg_free returns them.  Host pointers passed in are only read
 *     (or written, for outputs) during the call.
 *   - After HOTRG_EDEVICE or HOTRG_ENUMERIC, and after any failure inside a
 *     step that got past its argument checks (HOTRG_ENOMEM included), the
 *     context is marked failed: every later call except hotrg_free returns
 *     HOTRG_ESTATE.  The one exception is documented at hotrg_backward.
 */
#ifndef HOTRG_H
#define HOTRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HOTRG_OK = 0,
    HOTRG_EINVAL = -1,   /* bad argument (range, NULL pointer, axis not in 0..3) */
    HOTRG_ENOMEM = -2,   /* device allocation failed (allocator returned NULL) or mem_budget exceeded */
    HOTRG_EDEVICE = -3,  /* a HIP call failed */
    HOTRG_ESTATE = -4,   /* call not valid in the current state */
    HOTRG_ENUMERIC = -5  /* norm or trace not finite and positive (Tr <= 0 signals breakdown),
                            eigensolver not converged, non-finite derivative, or a
                            derivative through a cut with no spectral gap */
};

enum { HOTRG_FP64 = 0, HOTRG_BF16X3 = 1 };

typedef struct hotrg_ctx hotrg_ctx;

typedef struct {
    int precision;        /* HOTRG_FP64 or HOTRG_BF16X3 (split bf16 hi/lo, 3 products,
                             FP32 accumulation in chunks, FP64 across chunks) */
    int impurities;       /* 1: carry S_m (Eq. (2.11)) and S_e (Eq. (2.7)); 0: pure T only */
    int keep_checkpoints; /* 1: keep T^(k-1), U's and c_k of every step (needed by hotrg_backward) */
    int mixed_from_step;  /* first step (1-based) whose contraction uses the mixed path; 0 -> 4 */
    double tau_deg;       /* gap threshold of the degenerate-cut rule; 0 -> 1e-12 */
    void *stream;         /* hipStream_t; NULL = default stream */
    size_t slice_budget;  /* operand bytes of one K slice above which the contraction
                             slices also fix the b1' index (one value per slice); 0 ->
                             only where a slice would exceed 2^31 elements per tensor */
    int eig_max_sweeps;   /* sweep cap of the Jacobi eigensolver (0 -> 40, at most 1000); a
                             solve that reaches it with a squared off-diagonal norm above
                             1e-24 of the total fails the step with HOTRG_ENUMERIC */
    /* Device memory: when alloc is set, every buffer of the context comes from
     * alloc(bytes, alloc_ctx) (bytes a multiple of 256; the result must be device
     * memory aligned to 256 bytes, usable on `stream`) and goes back through
     * free(ptr, alloc_ctx) after the stream has finished with it.  alloc and free
     * are given together or not at all; NULL -> hipMalloc / hipFree.  A NULL
     * return from alloc gives HOTRG_ENOMEM. */
    void *(*alloc)(size_t bytes, void *alloc_ctx);
    void (*free)(void *ptr, void *alloc_ctx);
    void *alloc_ctx;
    size_t mem_budget;    /* most device bytes the context may hold at once; an allocation
                             that would exceed it fails with HOTRG_ENOMEM; 0 -> no limit */
    int dense_only;       /* 1: always contract densely; 0: at h = 0 use the Z2 block form
                             (below) whenever the state carries parity labels */
} hotrg_config;

/* Z2 block form of the contraction (h = 0).  At zero field Eq. (2.1) is
 * invariant under sigma -> -sigma, so every bond index carries a parity and
 * T, S_e are even, S_m odd: T^(0) from init has exact zeros on its odd
 * entries, and every isometry column of the FP64 eigensolver lies in one
 * parity sector (the Jacobi never rotates across an exactly zero block).  The
 * library tracks these labels (from init at h = 0, from hotrg_set_state when
 * the given tensors have exact zeros on the parity-violating entries with
 * bond parity i mod 2, and from the isometry columns after every step; a
 * column with non-zero rows of both parities drops the labels for the rest of
 * the flow).  A step with labels, other than the first step's S_e . S_e
 * pairing, contracts in blocks: per K slice the K indices of each parity class
 * meet only operand rows and columns of one class, so the product splits into
 * two GEMMs of about (M/2)(N/2)(K/2) -- a quarter of the dense work -- and
 * the output's parity-violating half is never formed.  Results equal the
 * dense contraction up to summation order. */

/* Set up the one-site state of Eqs. (2.2) and (2.6) with bond dimension 2:
 *   W = [[sqrt cosh b, sqrt sinh b], [sqrt cosh b, -sqrt sinh b]] (W W^T = bond matrix, Eq. (2.1)),
 *   T^(0) = sum_s e^{b h s} prod_8 W[s, i],  S^(0) = same with an extra factor s,
 * normalised by c_0 = |T^(0)|_F.  beta >= 0 (ferromagnetic), h finite, 1 <= dcut <= 13
 * (HOTRG_EINVAL otherwise): the environment matrices are at most dcut^2 x dcut^2, and the
 * eigensolver and adjoint kernels use LDS buffers sized for 169 rows.
 * hotrg_init uses the defaults (FP64, impurities on, no checkpoints). */
int hotrg_init(double beta, double h, int dcut, hotrg_ctx **out);
int hotrg_init_ex(double beta, double h, int dcut, const hotrg_config *cfg, hotrg_ctx **out);

/* One coarse-graining step along `axis` (Sec. 2; Eqs. (2.8)-(2.9) in 4D):
 * squeezed environments of the merged transverse legs (HOSVD, FP64), FP64
 * eigendecomposition on the device, truncation to k <= dcut, then
 * T' = U U U . T . T . U U U contracted on the MFMA cores, and S_m' = U.S_m.T.U,
 * S_e' = U.S_e.S_e.U on the first step and U.S_e.T.U afterwards.  All three
 * are divided by c_n = |T'|_F; ln Z bookkeeping is updated in FP64.
 * With the environment variable HOTRG_PROGRESS=1, long contractions (and
 * reverse steps of hotrg_backward) print about ten progress lines to stderr,
 * each after the device has finished the K slices it counts. */
int hotrg_step(hotrg_ctx *ctx, int axis);

/* ln Z / N after n steps (N = 2^n sites, Eqs. (2.3)-(2.5)):
 *   lnZ/N = sum_{k<=n} 2^-k ln c_k + 2^-n ln Tr T^(n). */
int hotrg_lnZ(hotrg_ctx *ctx, double *lnz_per_site);

typedef struct {
    int n;              /* steps taken */
    int dims[4];        /* current bond dimensions (D_x, D_y, D_z, D_t) */
    double lnz_per_site;
    double trace;       /* Tr T^(n) of the normalised tensor, Eq. (2.5) */
    double m_imp;       /* <sigma> = Tr S_m / Tr T, Eq. (2.12) */
    double nn_imp;      /* <sigma_i sigma_j> = Tr S_e / Tr T, Eq. (2.10); pair along the first step's axis */
    double e_imp;       /* -(1/N) dlnZ/dbeta estimate: -4 nn_imp - h m_imp */
    double X;           /* (Tr A)^2 / Tr A^2 along the last step's axis, Eqs. (3.2)-(3.3) */
    int last_axis;      /* axis of the last step, -1 before the first */
    int last_side[4];   /* per transverse axis: 0 backward / 1 forward env chosen; -1 untruncated or mu */
    int last_k[4];      /* kept dimension per axis in the last step */
    double last_eps[4]; /* discarded weight of the chosen side */
    double min_cut_gap; /* smallest (lam_k - lam_k+1)/lam_1 at a cut in the last step (inf if none) */
    int flagged;        /* 1 if a cut stayed inside a degenerate multiplet (no gap above tau) */
    double last_cn;     /* c_n of the last step (Frobenius norm before normalisation) */
    size_t device_bytes;/* device memory held by the context */
    int eig_sweeps;     /* most Jacobi sweeps one eigendecomposition of the last step took */
    double eig_residual;/* largest squared off-diagonal / total norm those solves left */
    int block_sparse;   /* 1 if the last step contracted in the Z2 block form (hotrg_config) */
} hotrg_obs;

/* Observables at the current step (impurity ratios need impurities = 1).
 * Unlike hotrg_lnZ this does not fail on Tr T <= 0 (possible for a state set
 * with hotrg_set_state): lnz_per_site is then NaN. */
int hotrg_observables(hotrg_ctx *ctx, hotrg_obs *out);

/* Per-site derivatives of ln Z / N at the current step (Sec. 2: the expectation
 * values follow from derivatives of ln Z, the route the paper sets beside the
 * impurity method and compares with it in Sec. 3), computed by reverse-mode
 * differentiation of the whole coarse-graining chain through the
 * eigendecomposition-derived isometries (needs keep_checkpoints = 1 and a flow
 * that started at hotrg_init):
 *   *dlnz_dbeta = d(lnZ/N)/d beta  (energy per site e = -dlnz_dbeta),
 *   *dlnz_dh    = d(lnZ/N)/d h     (magnetisation m = dlnz_dh / beta).
 * The c_n of Eq. (2.5)'s bookkeeping are held fixed (ln Z is exactly invariant
 * to them); an isometry's derivative keeps kept x discarded eigenvector pairs,
 * with weights 1 / (lam_i - lam_j).  Errors: HOTRG_EINVAL for beta <= 1e-3 (the
 * chain rule through sqrt(sinh b) diverges at 0); HOTRG_ESTATE without
 * checkpoints or after hotrg_set_state; HOTRG_ENUMERIC when a step's cut had no
 * spectral gap above tau (hotrg_obs.flagged; that derivative is undefined) --
 * returned before any device work and without marking the context failed -- or
 * when the result is not finite (context marked failed). */
int hotrg_backward(hotrg_ctx *ctx, double *dlnz_dbeta, double *dlnz_dh);

void hotrg_free(hotrg_ctx *ctx);
const char *hotrg_last_error(void);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * observables of hotrg_observables for device tensors the caller holds, with
 * no context and no allocation.  T (and S_m, S_e, both or neither) are device
 * pointers to rank-8 FP64 tensors of dims D_q in canonical leg order; `axis`
 * is the axis of X (Eqs. (3.2)-(3.3)); n and lnz_acc give lnZ/N = lnz_acc +
 * 2^-n ln Tr T; h enters e_imp.  out gets n, dims, lnz_per_site, trace, m_imp,
 * nn_imp, e_imp (NaN without impure tensors), X and last_axis = axis; the
 * decision fields are empty (last_side -1, min_cut_gap inf, the rest 0).
 * Work is enqueued on `stream` (hipStream_t, NULL = default) and the call
 * waits for it.  The trace kernel's partial results go to a fixed device
 * array of 3 + 13^2 doubles per GPU, owned by the library for the life of the
 * process: bond dimensions above 13 give HOTRG_EINVAL.  Calls that overlap on
 * one GPU (other threads, other streams) share that array and race; each call
 * overwrites every entry it reads.  Errors: HOTRG_EINVAL (arguments),
 * HOTRG_EDEVICE (a HIP call failed). */
int hotrg_observables_noalloc(const double *T, const double *Sm, const double *Se, const int dims[4], int axis,
                              double h, int n, double lnz_acc, void *stream, hotrg_obs *out);

/* ---- state access for parity tests and checkpoint/resume ------------------ */

/* Current dims and step count. */
int hotrg_get_dims(hotrg_ctx *ctx, int dims[4], int *n);

/* Copy tensor `which` (0 = T, 1 = S_m, 2 = S_e) to host memory `out`
 * (capacity `count` doubles; needs prod_q D_q^2 doubles). */
int hotrg_get_tensor(hotrg_ctx *ctx, int which, double *out, size_t count);

/* Replace the state by host tensors of dims `dims` (each D_q in 1..max(dcut,2)).
 * Sm or Se may be NULL when impurities are off.  `n` becomes the step count and
 * `lnz_acc` the accumulated sum_k 2^-k ln c_k. */
int hotrg_set_state(hotrg_ctx *ctx, const int dims[4], const double *T, const double *Sm,
                    const double *Se, int n, double lnz_acc);

/* The environment / eigendecomposition / cut stage of a step along `axis`
 * (Sec. 2; squeezed HOSVD environments, FP64 eigh, truncation to k <= dcut)
 * on the current state, without the contraction: the state and the step count
 * are unchanged.  Afterwards hotrg_get_isometry, hotrg_get_spectrum and the
 * last_side / last_k / last_eps / min_cut_gap / flagged / eig_* fields of
 * hotrg_observables describe this stage.  Used to check the stage on
 * identical inputs at sizes where a whole step is long. */
int hotrg_truncate(hotrg_ctx *ctx, int axis);

/* Step with caller-given isometries instead of the environment/eigh stage:
 * U[q] (host, row-major D_q^2 x k[q]) for the three transverse axes q != axis
 * (U[axis] is ignored).  Used to check the contraction on identical inputs. */
int hotrg_step_with_isometries(hotrg_ctx *ctx, int axis, const double *const U[4], const int k[4]);

/* Host copy of the isometry of axis `q` of the last step or hotrg_truncate
 * call (row-major, rows*cols doubles) and of the descending spectrum of its
 * (q, side) environment. */
int hotrg_get_isometry(hotrg_ctx *ctx, int q, double *out, size_t count, int *rows, int *cols);
int hotrg_get_spectrum(hotrg_ctx *ctx, int q, int side, double *out, size_t count, int *len);

/* Accumulated device time (ms, HIP events on the context stream) since the
 * last reset.  kernel 0: the contraction GEMM calls, one per K slice and
 * operand pairing (launches = their count, flops = 2 M N K summed); a bf16x3
 * call whose last round of output tiles is partly filled runs as a main
 * dispatch, a tail dispatch over that round split in k, and a small add.
 * kernel 1..3: the phases of hotrg_step, measured between events recorded at
 * its start, after the isometries (environments,
 * eigendecomposition, cut; Sec. 2), after the contraction (operand products
 * and GEMMs) and after the normalisation and permutation: 1 = isometries,
 * 2 = contraction (flops = the GEMM flops), 3 = normalisation; launches = steps
 * counted.  Phase times include device idle time while the host decides the
 * cut.  Querying a phase waits for the last step to finish.
 * kernel 4: launches = how many last isometry products of Z2 block-form
 * steps wrote their bf16 operand blocks through LDS tiles in whole 16-byte
 * pieces (the rest scatter element by element; the environment variable
 * HOTRG_Z2_TILE=0 selects that for every launch; both give identical bits);
 * ms = flops = 0.
 * kernel 5: launches = steps that hotrg_backward undid in the Z2 block form
 * (those whose forward contraction ran in it); ms = flops = 0. */
int hotrg_kernel_stats(hotrg_ctx *ctx, int kernel, double *ms, long long *launches, double *flops);
int hotrg_reset_stats(hotrg_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HOTRG_H */
