// Internal declarations shared by the HIP translation units of the HOTRG
// library.  Nothing here is part of the public ABI (include/hotrg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace hotrg {

// ---------------------------------------------------------------------------
// Division by a run-time constant without a hardware divide: for n < 2^31 and
// 1 <= d < 2^31, q = (umulhi(n, mul) + n) >> shift with
// shift = ceil(log2 d), mul = floor(2^32 (2^shift - d) / d) + 1
// (Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994).
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d, mul, shift;
};

inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.shift = s;
    f.mul = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
    return f;
}

__device__ __forceinline__ uint32_t fast_div(uint32_t n, const FastDiv &f) {
    return (__umulhi(n, f.mul) + n) >> f.shift;
}

// Isometry product with wave-uniform isometry addresses.  A thread owns one
// index of the `thread` dims (which address the input and the output) and
// loops over up to two `loop` dims that only address the isometry and the
// output:
//   out[o(t) + l1 o1 + l2 o2] = sum_{i < nsum} U[l1 u1 + l2 u2 + i us] * in[x(t) + i xs].
// The input run (nsum values) is loaded once per thread; every isometry load
// is the same for all lanes.  With o2 == 1 the l2 outputs of a thread are
// written as one contiguous run.
constexpr int XP_MAXD = 8;
constexpr int XP_MAXS = 16;
// With `pack` set (bf16 outputs only) the output offset o = r ld + k of a
// row-major operand is rewritten to the packed GEMM layout of
// launch_gemm_bf16x3 (pld = ld, pkb = ld / 32).
struct ExpandParams {
    int nd;
    int L1, L2, nsum;
    uint32_t threads;
    uint32_t u1, u2, o1, o2, xs, us;
    FastDiv ext[XP_MAXD];
    uint32_t in_st[XP_MAXD];
    uint32_t out_st[XP_MAXD];
    int pack;
    FastDiv pld;
    uint32_t pkb;
    uint32_t prow0;  // packed layout: row of the operand block where this launch's row 0 goes
    // Z2 block scatter (z2 = 1): the natural offset o = r zld + k of a
    // row-major operand slice is split into a row r and a K index k; the
    // tables give their parities (bit 31) and positions inside their parity
    // class.  An output with inner K parity i goes to block i, GEMM class
    // g = i ^ zs; it is structurally zero (not written) unless the row's
    // parity is zP ^ g.  Block i gets row zrow_off[g] + position, column the
    // K position; FP64 blocks are row-major with row length zld_out[i], bf16
    // blocks packed with zpkb[i] = zld_out[i] / 32 k blocks per row tile.
    int z2;
    // z2 == 4: the transposed scatter of the reverse pass (see
    // iso_expand_z2t_kernel; zrs = K step of the second loop).
    // z2 == 2: the run form (see iso_expand_z2run_kernel): the first loop
    // steps whole rows (o1 = zrs * zld), the second stays inside the row
    // (o2 < zld and no carry out of the K part), so a thread needs one row
    // and N K lookups
    uint32_t zrs;
    int zpair;  // run form, bf16: the second loop steps one K position (o2 == 1), so
                // consecutive outputs of a run may go out as 4-byte pairs
    // z2 == 3: the tile form (bf16 only, see iso_expand_z2tile_kernel).  The
    // thread dims are [K-outer | row | inner]: a unit is one multi-index of
    // the K-outer and row dims with its tP inner threads; a K group (one
    // K-outer multi-index) covers the natural K run [K0, K0 + tnK) through
    // the inner dims and the second loop, and a unit covers L1 consecutive
    // rows (first loop, one row per step).  A tile is tupb consecutive units
    // of one K group: a rectangle of natural rows x K indices whose outputs
    // are gathered in LDS in class order and written as whole 16-byte pieces.
    uint32_t tP, tNRP, tKg, tupb, tnK;
    uint32_t tLD;     // LDS row length of a tile (bf16 elements, multiple of 8)
    uint32_t tslots;  // thread slots per unit (a multiple of 64)
    const uint32_t *tperm;  // slot -> inner thread (~0u: idle), K-run parity 0 first
    const double *tU;       // the isometry block as [l1][l2][j], j < tNH (see the kernel)
    int tNH;                // compacted summed-index count (z2tile_nh)
    uint32_t tlab1, tlab2;  // parity labels of the loop indices l1, l2 (bit l = label of index l)
    uint64_t tI[2];         // summed indices of parity 0 / 1, 4 bits each in order
    uint32_t tnI[2];        // their counts
    uint32_t zKc[2];  // K indices of each class (size of ktab = zKc[0] + zKc[1])
    uint32_t zNr[2];  // rows of each parity (size of rtab = zM)
    uint32_t zM;
    FastDiv zld;
    const uint32_t *rtab, *ktab;
    uint32_t zs, zP;
    uint32_t zrow_off[2];
    uint32_t zld_out[2], zpkb[2];
    double *zout[2];
    uint16_t *zhi[2], *zlo[2];
};

// Z2 parity class tables: bit 31 = parity, low 31 bits = position of the
// index within its class (natural order).
constexpr uint32_t Z2_PAR = 0x80000000u;
// dynamic LDS of one z2 tile workgroup: the hi and lo tiles
inline size_t z2tile_lds_bytes(const ExpandParams &p) {
    return (size_t)2 * p.tupb * p.L1 * p.tLD * sizeof(uint16_t);
}
constexpr size_t Z2TILE_MAX_LDS = 64 * 1024;
constexpr int Z2TILE_MAX_THREADS = 512;

// Generic contraction of two strided views (reverse pass):
//   out[z(o)] (+)= alpha * sum_s X[x(o) + x(s)] * Y[y(o) + y(s)]
// o runs over `ndo` output dims (row-major), s over `nds` summed dims.
constexpr int EIN_MAXO = 10;
constexpr int EIN_MAXS = 8;
struct EinsumParams {
    int ndo, nds;
    uint32_t nout, S, chunk, nchunks;
    FastDiv oext[EIN_MAXO];
    uint32_t ox[EIN_MAXO], oy[EIN_MAXO], oz[EIN_MAXO];
    uint32_t sext[EIN_MAXS], sx[EIN_MAXS], sy[EIN_MAXS];
    double alpha;
    int accumulate;
};

// Outer-product reduction of the reverse pass (a contraction whose every
// output index addresses only one operand):
//   out[zm(m) + zn(n)] (+)= alpha * sum_k X[x(k) + xm(m)] * Y[y(k) + yn(n)],
// m over ndm dims (extents mext, strides mx in X, mz in out), n over ndn dims
// (next, ny, nz), k over nds dims (sext, sx, sy), each row-major.  Mo = prod
// mext, No = prod next (Mo No <= 4096).  xmfast / ynfast: stage X (Y) with m
// (n) as the fastest index (else k).
constexpr int RED_MAXD = 4;
struct RedParams {
    int ndm, ndn, nds;
    uint32_t mext[RED_MAXD], mx[RED_MAXD], mz[RED_MAXD];
    uint32_t next[RED_MAXD], ny[RED_MAXD], nz[RED_MAXD];
    FastDiv sext[EIN_MAXS];
    uint32_t sx[EIN_MAXS], sy[EIN_MAXS];
    FastDiv mo, no;
    uint32_t S, chunk, nchunks;
    int xmfast, ynfast;
    double alpha;
    int accumulate;
};

// Small matrix times many strided columns (reverse pass): a contraction whose
// summed indices k address both operands and whose output indices split into
// X-only indices m (ndm dims, M <= 256 values) and Y-only indices n (ndn dims):
//   out[zm(m) + zn(n)] (+)= alpha * sum_k X[xm(m) + xk(k)] * Y[yn(n) + yk(k)],
// K = prod sext <= 100 (all rows of the multi-indices row-major).
constexpr int XMV_MAXM = 256;
struct XmvParams {
    int ndm, ndn, nds;
    uint32_t mext[RED_MAXD], mx[RED_MAXD], mz[RED_MAXD];
    FastDiv next[EIN_MAXO];
    uint32_t ny[EIN_MAXO], nz[EIN_MAXO];
    uint32_t sext[EIN_MAXS], sx[EIN_MAXS], sy[EIN_MAXS];
    uint32_t M, N, K;
    double alpha;
    int accumulate;
};

// Adjoint of the last isometry product of one K slice, fused with the
// adjoint of that isometry (one pass over the operand adjoint X):
//   out[o, j, l]    = sum_{c, s} U[l, s, c] X[o, j, c, s]
//   Ubar[l, s, c] += sum_{o, j} Y[o, j, l] X[o, j, c, s]
// with o = (o1, o2), offsets  X: o1 x_o1 + o2 x_o2 + j xj + c xc + s xs,
// out / Y: o1 out_o1 + o2 out_o2 + j oj + l ol,  U / Ubar: l ul + s us + c uc;
// c < L, s, l < N.  Element offsets below 2^32.
struct LastProdParams {
    uint32_t n_o1, n_o2, NJ;
    uint32_t x_o1, x_o2, xj, xc, xs;
    uint32_t out_o1, out_o2, oj, ol;
    uint32_t ul, us, uc;
    int L, N;
    // cls: X is given in Z2 class blocks instead (reverse pass, block form):
    // the natural offset o of an X entry splits into the row r = o / ks and
    // the K index k = o - r ks; the entry is blk[b][pos(r) ldb[b] + pos(k)]
    // (b = class of k in ktab) when the parity of r (rtab) is b ^ zs, else 0
    int cls;
    const double *blk[2];
    uint32_t ldb[2];
    const uint32_t *rtab, *ktab;
    uint32_t zs;
    FastDiv ks;
};

constexpr int PERM_MAXD = 8;
struct PermParams {
    int nd;
    uint32_t total;
    FastDiv ext[PERM_MAXD];
    uint32_t in_st[PERM_MAXD];
};

// ---- launchers (all asynchronous on `s`) ----------------------------------
void launch_init_site(double *T, double *S, double w00, double w01, double w10, double w11,
                      double v_up, double v_dn, hipStream_t s);
void launch_permute(const PermParams &p, const double *in, double *out, double scale, hipStream_t s);
// Reverse pass, Z2 block form (pure T): C_bar class blocks C_g (N_g x N_g,
// C_0 then C_1, row-major) and their transposes from Tbar; inv lists the
// natural GEMM rows of class 0 then class 1, roff / coff give a row's / a
// column's offset in Tbar.
void launch_z2_cbar(const double *Tbar, const uint32_t *inv, const uint32_t *roff, const uint32_t *coff,
                    uint32_t N0, uint32_t N1, double scale, double *Cg, double *CgT, hipStream_t s);
// class-block GEMM outputs (block b: rows = class positions of the rows, row
// length ldb) -> natural R x Ks operand adjoint with exact zeros elsewhere
void launch_z2_unscatter(const double *b0, const double *b1, uint32_t ld0, uint32_t ld1, const uint32_t *rtab,
                         const uint32_t *ktab, uint32_t zs, uint32_t zP, uint32_t Ks, uint32_t R, double *out,
                         hipStream_t s);
// dst[j] = src[idx[j]], or 0 where idx[j] < 0, for j < n
void launch_gather_or_zero(const double *src, const int32_t *idx, double *dst, int n, hipStream_t s);
// compacted summed-index count the z2 tile kernel is compiled for, given the
// larger parity class nmax of an N-value summed index (N when no split fits)
int z2tile_nh(int N, int nmax);
// out (FP64) or hi/lo (bf16 split) when hi != nullptr
void launch_iso_expand(const ExpandParams &p, const double *in, const double *U, double *out,
                       uint16_t *hi, uint16_t *lo, hipStream_t s);
// sum of squares of x[0..n) -> *out (device), deterministic two-pass reduction
void launch_sumsq(const double *x, size_t n, double *partials, int npartials, double *out,
                  hipStream_t s);
// traces of up to 3 tensors with dims D[4] (legs x x' y y' z z' t t') and the
// A matrix of Eq. (3.2) along `axis` of the first tensor.  out[0..2] traces,
// out[3..3+D_axis^2) the A matrix.
void launch_trace_obs(const double *T0, const double *T1, const double *T2, const int D[4],
                      int axis, double *out, hipStream_t s);
// G[(p, q), (p', q')] = sum_r X[p q r] X[p' q' r] for X given as R x K row-major
// (R <= 288): split-K partials then a fixed-order reduction.
void launch_gram(const double *X, int R, size_t K, double *partials, int nchunks, double *G,
                 hipStream_t s);
// E[(p, q), (p', q')] = sum_{a, a'} G1[p a p' a'] G2[q a q' a']
void launch_env_combine(const double *G1, const double *G2, int Dp, int Dq, int Da, double *E,
                        hipStream_t s);
void launch_identity(double *U, int n, hipStream_t s);
void launch_zero(double *x, size_t n, hipStream_t s);
// X[R][K] (FP64, row stride K) -> bf16 hi / lo splits in the packed layout of
// launch_gemm_bf16x3 with row length ld (a multiple of 64, >= K; padding
// columns written as zero).  R * ld < 2^32.
void launch_split_pack(const double *X, uint32_t R, uint32_t K, uint32_t ld, uint16_t *hi, uint16_t *lo,
                       hipStream_t s);

// Z2 block form of the step's output -> canonical tensors.  C_g (g = 0, 1)
// holds, for GEMM class g, rows [T rows of parity g | S_m rows of parity 1-g |
// S_e rows of parity g] (positions from rtab) by the columns of parity g, row
// length N_g.  Output element o of tensor t (canonical order of the new dims)
// has row index sum_l digit_l rst[l] and column index sum_l digit_l cst[l];
// entries whose row and column parities differ from the tensor's parity
// (even T, S_e; odd S_m) are exact zeros.  out = scale * C value.
struct Z2UnpackParams {
    int nd;
    uint32_t total;
    FastDiv ext[PERM_MAXD];
    uint32_t rst[PERM_MAXD], cst[PERM_MAXD];
    const uint32_t *rtab;
    const double *C[2];
    uint32_t N[2];
    uint32_t row_off[2];  // this tensor's first row in C_g
    uint32_t P;           // tensor parity
};
void launch_z2_unpack(const Z2UnpackParams &p, double *out, double scale, hipStream_t s);

// reverse pass (kernels_adjoint.hip)
// LastProdParams contraction; partial: (n_o1 * n_o2 + 64) * L * N * N doubles
// (per-workgroup sums, then 64 group sums), added into Ubar in a fixed order.  Returns false (and
// launches nothing) if N is not one of the compiled sizes (2 .. 12) or L > 16.
bool launch_lastprod_adjoint(const LastProdParams &p, const double *X, const double *Y, const double *U,
                             double *out, double *Ubar, double *partial, hipStream_t s);
void launch_einsum(EinsumParams p, const double *X, const double *Y, double *out, double *partial,
                   size_t partial_cap, hipStream_t s);
// RedParams contraction; false (nothing launched) when the outputs exceed
// 4096, the LDS staging exceeds 64 KB or the partial buffer cannot hold one
// chunk per output
bool launch_red(RedParams p, const double *X, const double *Y, double *out, double *partial, size_t partial_cap,
                hipStream_t s);
// XmvParams contraction (X gathered into xc, capacity xc_cap doubles); false
// (nothing launched) when K > 100, M > 256 or xc is too small
bool launch_xmv(const XmvParams &p, const double *X, const double *Y, double *out, double *xc, size_t xc_cap,
                hipStream_t s);
void launch_eigh_adjoint(const double *V, const double *lam, const double *Ubar, int n, int k, double *Ebar,
                         hipStream_t s);
void launch_diag_set(double *T, const int D[4], const uint32_t diag_st[4], double value, hipStream_t s);
void launch_site_dot(const double *Tbar, double wc, double ws, double dwc, double dws, double beta, double h,
                     double vu, double vd, double inv_c0, double *out, hipStream_t s);

// Jacobi eigensolver: `count` symmetric n x n matrices (n <= 169) at A + i*n*n,
// eigenvalues (descending) to lam + i*n, eigenvectors as columns of V + i*n*n
// (row-major, V[r*n + j] = component r of vector j).  work: 2*count*n*n doubles.
// At most max_sweeps sweeps; sweeps[i] gets the number taken and resid[i] the
// squared off-diagonal norm left divided by the squared Frobenius norm.
void launch_jacobi_eigh(const double *A, int n, int count, double *lam, double *V, double *work,
                        int *sweeps, double *resid, int max_sweeps, hipStream_t s);

// C[M x N] (ldc) (+)= A[M x K] (lda) * B[N x K]^T (ldb); FP64 MFMA.
void launch_gemm_f64(const double *A, const double *B, double *C, int M, int N, int K, size_t lda,
                     size_t ldb, size_t ldc, int accumulate, hipStream_t s);
// Same product from bf16 hi/lo splits: A ~ Ah + Al, B ~ Bh + Bl; computes
// Ah Bh^T + Ah Bl^T + Al Bh^T with FP32 MFMA accumulation over chunks of at
// most 32768 k, summed in FP64.  Operands are in the packed layout below; A
// stacks ntA tensors of M rows each (C rows t M + r), B has N rows; K is a
// multiple of 64.
//
// Packed layout of an operand with R rows and K columns (K a multiple of
// 32): rows are padded to Rp = roundup(R, 256); element (r, k) sits at
//   ((r / 256) (K / 32) + k / 32) 8192 + (r % 256) 32 + k % 32,
// i.e. every 256 x 32 block the GEMM stages at once is one contiguous run.
constexpr int PACK_ROWS = 256, PACK_K = 32;
__host__ __device__ inline size_t packed_offset(size_t r, size_t k, size_t K) {
    return ((r / PACK_ROWS) * (K / PACK_K) + k / PACK_K) * (PACK_ROWS * PACK_K) + (r % PACK_ROWS) * PACK_K +
           k % PACK_K;
}
inline size_t packed_rows(size_t R) { return (R + PACK_ROWS - 1) / PACK_ROWS * PACK_ROWS; }
// `part` (may be null): scratch for the second k-halves of the last, partly
// filled round of tiles, GEMM_TAIL_MAX_TILES blocks of 256 x 256 doubles.
constexpr int GEMM_TAIL_MAX_TILES = 128;
// Several independent bf16x3 products (at most two) in one launch: their
// tiles form one list, so the chip is filled by the tiles of both and only
// the last round of the combined list is partly filled.
struct X3Gemm {
    const uint16_t *Ah, *Al, *Bh, *Bl;
    double *C;
    int M, ntA, N, K;
    size_t ldc;
    int accumulate;
};
void launch_gemm_bf16x3_multi(const X3Gemm *g, int count, hipStream_t s, double *part);
void launch_gemm_bf16x3(const uint16_t *Ah, const uint16_t *Al, const uint16_t *Bh, const uint16_t *Bl,
                        double *C, int M, int ntA, int N, int K, size_t ldc, int accumulate, hipStream_t s,
                        double *part);

}  // namespace hotrg
