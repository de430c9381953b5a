// Kernels of the reverse-mode pass (adjoint of the coarse-graining chain).
//
// * einsum_kernel: a generic two-operand contraction over strided views,
//     out[z(o)] (+)= alpha * sum_s X[x(o) + x(s)] * Y[y(o) + y(s)],
//   with the summed multi-index s walked as an odometer (one division per
//   thread) and optionally split into chunks whose partial sums are added in a
//   fixed order (deterministic).  Every adjoint of an isometry product, of an
//   isometry itself, of the environment combination and of the Grams is one
//   such contraction; the host sends the two shapes that dominate the reverse
//   pass to dedicated kernels instead (red_kernel: few outputs, long sums;
//   xmv_kernel: a small matrix times many strided columns).
// * lastprod_adjoint_kernel: the adjoint of the last isometry product of a K
//   slice fused with that isometry's adjoint, reading the operand adjoint in
//   the natural layout or in Z2 class blocks.
// * eigh_adjoint_kernel: E_bar = sym(V_perp (F o (V_perp^T U_bar)) U^T) with
//   F[j, i] = 1 / (lam_i - lam_j) for kept i and discarded j -- the derivative
//   of the kept eigenvectors restricted to kept x discarded pairs (rotations
//   inside the kept space are gauge and do not change any trace).
// * seed and final contraction with dT^(0)/d(beta, h).
#include "hotrg_internal.h"

#include <algorithm>

namespace hotrg {

namespace {
constexpr int kT = 256;
}

__global__ void __launch_bounds__(kT) einsum_kernel(EinsumParams p, const double *__restrict__ X,
                                                    const double *__restrict__ Y, double *__restrict__ out,
                                                    double *__restrict__ partial) {
    const uint32_t ch = blockIdx.y;
    for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < p.nout; o += gridDim.x * blockDim.x) {
        uint32_t rem = o, xb = 0, yb = 0, zb = 0;
        for (int k = p.ndo - 1; k >= 0; --k) {
            uint32_t q = fast_div(rem, p.oext[k]);
            uint32_t c = rem - q * p.oext[k].d;
            xb += c * p.ox[k];
            yb += c * p.oy[k];
            zb += c * p.oz[k];
            rem = q;
        }
        const uint32_t s0 = ch * p.chunk;
        const uint32_t s1 = (p.S - s0 < p.chunk) ? p.S : s0 + p.chunk;
        double acc = 0.0;
        if (s0 < p.S) {
            uint32_t cs[EIN_MAXS];
            uint32_t xo = 0, yo = 0, r = s0;
#pragma unroll
            for (int k = EIN_MAXS - 1; k >= 0; --k) {
                cs[k] = 0;
                if (k < p.nds) {
                    cs[k] = r % p.sext[k];
                    r /= p.sext[k];
                    xo += cs[k] * p.sx[k];
                    yo += cs[k] * p.sy[k];
                }
            }
            for (uint32_t s = s0; s < s1; ++s) {
                acc = fma(X[xb + xo], Y[yb + yo], acc);
#pragma unroll
                for (int k = EIN_MAXS - 1; k >= 0; --k) {
                    if (k >= p.nds) continue;
                    cs[k] += 1;
                    xo += p.sx[k];
                    yo += p.sy[k];
                    if (cs[k] < p.sext[k]) break;
                    cs[k] = 0;
                    xo -= p.sext[k] * p.sx[k];
                    yo -= p.sext[k] * p.sy[k];
                }
            }
        }
        if (p.nchunks == 1) {
            const double v = p.alpha * acc;
            out[zb] = p.accumulate ? out[zb] + v : v;
        } else {
            partial[(size_t)ch * p.nout + o] = acc;
        }
    }
}

__global__ void __launch_bounds__(kT) einsum_reduce_kernel(EinsumParams p, const double *__restrict__ partial,
                                                           double *__restrict__ out) {
    for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < p.nout; o += gridDim.x * blockDim.x) {
        uint32_t rem = o, zb = 0;
        for (int k = p.ndo - 1; k >= 0; --k) {
            uint32_t q = fast_div(rem, p.oext[k]);
            zb += (rem - q * p.oext[k].d) * p.oz[k];
            rem = q;
        }
        double acc = 0.0;
        for (uint32_t c = 0; c < p.nchunks; ++c) acc += partial[(size_t)c * p.nout + o];
        const double v = p.alpha * acc;
        out[zb] = p.accumulate ? out[zb] + v : v;
    }
}

void launch_einsum(EinsumParams p, const double *X, const double *Y, double *out, double *partial,
                   size_t partial_cap, hipStream_t s) {
    if (p.nout == 0) return;
    // enough threads to fill the chip: split long sums when there are few outputs
    uint32_t want = p.nout >= (1u << 18) ? 1u : (uint32_t)(((1u << 18) + p.nout - 1) / p.nout);
    uint32_t maxc = p.S / 64 > 0 ? p.S / 64 : 1;
    uint32_t nch = want < maxc ? want : maxc;
    if (nch > 4096) nch = 4096;
    while (nch > 1 && (size_t)nch * p.nout > partial_cap) nch /= 2;
    if (nch < 1) nch = 1;
    p.nchunks = nch;
    p.chunk = (p.S + nch - 1) / nch;
    uint32_t gx = (p.nout + kT - 1) / kT;
    if (gx > 65535) gx = 65535;
    einsum_kernel<<<dim3(gx, nch), kT, 0, s>>>(p, X, Y, out, partial);
    if (nch > 1) einsum_reduce_kernel<<<gx, kT, 0, s>>>(p, partial, out);
}

// ---------------------------------------------------------------------------
// Outer-product reduction (see RedParams): the contractions whose outputs are
// few and whose sums are long (the isometry adjoints, D^2 k outputs over D^6
// or D^7 terms).  Workgroup c walks the summed range [c chunk, (c+1) chunk)
// in blocks of RED_KB indices: the block's rows of X (RED_KB x Mo) and of Y
// (RED_KB x No) are staged in LDS with coalesced loads (the operand's
// contiguous index fastest), then each thread adds the block's terms of its
// outputs in k order; the workgroup's partial sums go to `partial`, which
// red_finish_kernel adds in chunk order (deterministic).
// ---------------------------------------------------------------------------
namespace {
constexpr int RED_KB = 32;
constexpr int RED_MAXO = 16;  // outputs per thread: Mo No <= 16 * 256
}  // namespace

__global__ void __launch_bounds__(kT) red_kernel(RedParams p, const double *__restrict__ X,
                                                 const double *__restrict__ Y, double *__restrict__ partial) {
    extern __shared__ __align__(16) double rsm[];
    const uint32_t Mo = p.mo.d, No = p.no.d, nout = Mo * No;
    double *Xs = rsm;                    // [RED_KB][Mo]
    double *Ys = Xs + RED_KB * Mo;       // [RED_KB][No]
    uint32_t *xk = (uint32_t *)(Ys + RED_KB * No);
    uint32_t *yk = xk + RED_KB;
    uint32_t *xmo = yk + RED_KB;         // [Mo]
    uint32_t *yno = xmo + Mo;            // [No]
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < Mo; i += blockDim.x) {
        uint32_t r = i, o = 0;
        for (int d = p.ndm - 1; d >= 0; --d) {
            o += (r % p.mext[d]) * p.mx[d];
            r /= p.mext[d];
        }
        xmo[i] = o;
    }
    for (uint32_t i = tid; i < No; i += blockDim.x) {
        uint32_t r = i, o = 0;
        for (int d = p.ndn - 1; d >= 0; --d) {
            o += (r % p.next[d]) * p.ny[d];
            r /= p.next[d];
        }
        yno[i] = o;
    }
    double acc[RED_MAXO];
#pragma unroll
    for (int j = 0; j < RED_MAXO; ++j) acc[j] = 0.0;
    const uint32_t k0 = blockIdx.x * p.chunk;
    const uint32_t k1 = min(p.S, k0 + p.chunk);
    for (uint32_t kb0 = k0; kb0 < k1; kb0 += RED_KB) {
        const uint32_t nk = min((uint32_t)RED_KB, k1 - kb0);
        __syncthreads();  // previous block consumed (and the offset tables written)
        if (tid < nk) {
            uint32_t r = kb0 + tid, xo = 0, yo = 0;
            for (int d = p.nds - 1; d >= 0; --d) {
                const uint32_t q = fast_div(r, p.sext[d]);
                const uint32_t c = r - q * p.sext[d].d;
                xo += c * p.sx[d];
                yo += c * p.sy[d];
                r = q;
            }
            xk[tid] = xo;
            yk[tid] = yo;
        }
        __syncthreads();
        for (uint32_t e = tid; e < RED_KB * Mo; e += blockDim.x) {
            uint32_t kk, m;
            if (p.xmfast) {
                kk = fast_div(e, p.mo);
                m = e - kk * Mo;
            } else {
                m = e / RED_KB;
                kk = e % RED_KB;
            }
            if (kk < nk) Xs[kk * Mo + m] = X[xk[kk] + xmo[m]];
        }
        for (uint32_t e = tid; e < RED_KB * No; e += blockDim.x) {
            uint32_t kk, n;
            if (p.ynfast) {
                kk = fast_div(e, p.no);
                n = e - kk * No;
            } else {
                n = e / RED_KB;
                kk = e % RED_KB;
            }
            if (kk < nk) Ys[kk * No + n] = Y[yk[kk] + yno[n]];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RED_MAXO; ++j) {
            const uint32_t e = tid + j * blockDim.x;
            if (e >= nout) break;
            const uint32_t m = fast_div(e, p.no), n = e - m * No;
            double a = acc[j];
            for (uint32_t kk = 0; kk < nk; ++kk) a = fma(Xs[kk * Mo + m], Ys[kk * No + n], a);
            acc[j] = a;
        }
    }
#pragma unroll
    for (int j = 0; j < RED_MAXO; ++j) {
        const uint32_t e = tid + j * blockDim.x;
        if (e < nout) partial[(size_t)blockIdx.x * nout + e] = acc[j];
    }
}

__global__ void __launch_bounds__(kT) red_finish_kernel(RedParams p, const double *__restrict__ partial,
                                                        double *__restrict__ out) {
    const uint32_t Mo = p.mo.d, No = p.no.d, nout = Mo * No;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nout; e += gridDim.x * blockDim.x) {
        const uint32_t m = fast_div(e, p.no), n = e - m * No;
        uint32_t z = 0, r = m;
        for (int d = p.ndm - 1; d >= 0; --d) {
            z += (r % p.mext[d]) * p.mz[d];
            r /= p.mext[d];
        }
        r = n;
        for (int d = p.ndn - 1; d >= 0; --d) {
            z += (r % p.next[d]) * p.nz[d];
            r /= p.next[d];
        }
        double a = 0.0;
        for (uint32_t c = 0; c < p.nchunks; ++c) a += partial[(size_t)c * nout + e];
        const double v = p.alpha * a;
        out[z] = p.accumulate ? out[z] + v : v;
    }
}

size_t red_lds_bytes(const RedParams &p) {
    return (size_t)RED_KB * (p.mo.d + p.no.d) * sizeof(double) + (size_t)(2 * RED_KB + p.mo.d + p.no.d) * 4;
}

bool launch_red(RedParams p, const double *X, const double *Y, double *out, double *partial, size_t partial_cap,
                hipStream_t s) {
    const size_t nout = (size_t)p.mo.d * p.no.d;
    if (nout == 0 || nout > (size_t)RED_MAXO * kT || p.S == 0 || red_lds_bytes(p) > 64 * 1024) return false;
    size_t nch = std::min<size_t>((p.S + 1023) / 1024, 2048);
    nch = std::min(nch, partial_cap / nout);
    if (nch < 1) return false;
    uint32_t chunk = (uint32_t)((p.S + nch - 1) / nch);
    chunk = (chunk + RED_KB - 1) / RED_KB * RED_KB;
    p.chunk = chunk;
    p.nchunks = (p.S + chunk - 1) / chunk;
    red_kernel<<<p.nchunks, kT, red_lds_bytes(p), s>>>(p, X, Y, partial);
    red_finish_kernel<<<(uint32_t)((nout + kT - 1) / kT), kT, 0, s>>>(p, partial, out);
    return true;
}

// ---------------------------------------------------------------------------
// Small-matrix products over many strided columns (see XmvParams): the
// adjoints of the isometry products and of the Grams, where a small matrix
// X (M x K, K <= 100) multiplies D^6..D^8 strided columns of Y.  One thread
// per column n keeps the column's K values in registers; X is first gathered
// into a dense M x KMAX array (zero past K) so that the product reads it
// through wave-uniform addresses (scalar loads).
// ---------------------------------------------------------------------------
__global__ void xmv_gather_kernel(XmvParams p, const double *__restrict__ X, double *__restrict__ Xc, int kmax) {
    const uint32_t M = p.M;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < M * (uint32_t)kmax; e += gridDim.x * blockDim.x) {
        const uint32_t m = e / (uint32_t)kmax, k = e - m * (uint32_t)kmax;
        double v = 0.0;
        if (k < p.K) {
            uint32_t o = 0, r = m;
            for (int d = p.ndm - 1; d >= 0; --d) {
                o += (r % p.mext[d]) * p.mx[d];
                r /= p.mext[d];
            }
            r = k;
            for (int d = p.nds - 1; d >= 0; --d) {
                o += (r % p.sext[d]) * p.sx[d];
                r /= p.sext[d];
            }
            v = X[o];
        }
        Xc[e] = v;
    }
}

template <int KMAX>
__global__ void __launch_bounds__(kT) xmv_kernel(XmvParams p, const double *__restrict__ Xc,
                                                 const double *__restrict__ Y, double *__restrict__ out) {
    __shared__ uint32_t yk[KMAX];
    __shared__ uint32_t zmo[XMV_MAXM];
    for (uint32_t k = threadIdx.x; k < KMAX; k += blockDim.x) {
        uint32_t o = 0, r = k;
        if (k < p.K)
            for (int d = p.nds - 1; d >= 0; --d) {
                o += (r % p.sext[d]) * p.sy[d];
                r /= p.sext[d];
            }
        yk[k] = o;
    }
    for (uint32_t m = threadIdx.x; m < p.M; m += blockDim.x) {
        uint32_t o = 0, r = m;
        for (int d = p.ndm - 1; d >= 0; --d) {
            o += (r % p.mext[d]) * p.mz[d];
            r /= p.mext[d];
        }
        zmo[m] = o;
    }
    __syncthreads();
    for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += gridDim.x * blockDim.x) {
        uint32_t rem = n, yb = 0, zb = 0;
        for (int d = p.ndn - 1; d >= 0; --d) {
            const uint32_t q = fast_div(rem, p.next[d]);
            const uint32_t c = rem - q * p.next[d].d;
            yb += c * p.ny[d];
            zb += c * p.nz[d];
            rem = q;
        }
        double y[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) y[k] = Y[yb + yk[k]];  // (k >= K: offset 0, met by a zero of Xc)
        for (uint32_t m = 0; m < p.M; ++m) {
            const double *xm = Xc + (size_t)m * KMAX;
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) acc = fma(xm[k], y[k], acc);
            double *o = out + zb + zmo[m];
            const double v = p.alpha * acc;
            *o = p.accumulate ? *o + v : v;
        }
    }
}

bool launch_xmv(const XmvParams &p, const double *X, const double *Y, double *out, double *xc, size_t xc_cap,
                hipStream_t s) {
    int kmax = p.K <= 16 ? 16 : (p.K <= 36 ? 36 : (p.K <= 64 ? 64 : (p.K <= 100 ? 100 : 0)));
    if (kmax == 0 || p.M == 0 || p.M > XMV_MAXM || p.N == 0 || (size_t)p.M * kmax > xc_cap) return false;
    const uint32_t ng = (uint32_t)std::min<size_t>(((size_t)p.M * kmax + kT - 1) / kT, 1024);
    xmv_gather_kernel<<<ng, kT, 0, s>>>(p, X, xc, kmax);
    const uint32_t g = (uint32_t)std::min<size_t>(((size_t)p.N + kT - 1) / kT, 65535);
    switch (kmax) {
        case 16: xmv_kernel<16><<<g, kT, 0, s>>>(p, xc, Y, out); break;
        case 36: xmv_kernel<36><<<g, kT, 0, s>>>(p, xc, Y, out); break;
        case 64: xmv_kernel<64><<<g, kT, 0, s>>>(p, xc, Y, out); break;
        default: xmv_kernel<100><<<g, kT, 0, s>>>(p, xc, Y, out); break;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Fused adjoint of the last isometry product of a K slice (see
// LastProdParams).  Workgroup (o1, o2) walks j in tiles of JT: the tile of X
// (JT x L N, row (j) by (c, s)) and of Y (JT x N) is staged in LDS, and both
// products of the tile are small dense matrix products on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64):
//   outputs    D[j, l]   = sum_cs X[j, cs] U[l, cs]   (16 j x 16 l blocks),
//   isometry   E[l, cs] += sum_j Y[j, l] X[j, cs]      (16 l x 16 cs blocks,
//              accumulated over the tiles in the matrix registers);
// at the end the workgroup stores E as one row of `partial`.  The products
// take a small part of the time (the element-wise form of the same sums, three
// LDS operands per four FMAs, was about 1.5% slower in the whole reverse
// pass); the kernel is bound by the gather of X, through the class tables in
// the block form.
// MFMA operand layout (16 x 4 A, 4 x 16 B, 16 x 16 D): lane t
// supplies A[t % 16][t / 16] and B[t / 16][t % 16], and holds D[4 i + t / 16]
// [t % 16] in its register i.
// ---------------------------------------------------------------------------
namespace {
constexpr int LP_JT = 32;
constexpr int LP_MAXL = 16;
constexpr int LP_UPT = 9;  // L N N <= 16 * 12 * 12 = 2304 = 256 * 9 isometry-adjoint entries
constexpr int LP_MAXB = 3;  // 16-column blocks of E per wave: L N <= 192 = 12 blocks over 4 waves
typedef double lp_dbl4 __attribute__((ext_vector_type(4)));

// LDS row length of the X / U tiles: L N rounded up to whole 4-column MFMA
// steps, plus one (an odd stride spreads the 16 rows of an operand read over
// the banks); the padding columns hold zeros.  (Kept short: at 4 workgroups
// per CU the usual grid of one slice, 1000 workgroups, runs in one round.)
__host__ __device__ inline int lp_stride(int L, int N) { return (L * N + 3) / 4 * 4 + 1; }
}  // namespace

// (four waves per SIMD: four workgroups per CU, so the usual 1000-workgroup
// grid of one slice runs in one round)
template <int N>
__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(4)))
lastprod_adjoint_kernel(LastProdParams p, const double *__restrict__ X, const double *__restrict__ Y,
                        const double *__restrict__ U, double *__restrict__ out, double *__restrict__ partial) {
    static_assert(N <= 16, "one 16-wide block of l");
    extern __shared__ __align__(16) double lp_sm[];
    const int L = p.L, LN = L * N;
    const int SX = lp_stride(L, N);
    const int NB = (LN + 15) / 16;     // 16-column blocks of E
    const int KP = (LN + 3) / 4 * 4;   // k extent of the output products (< SX)
    double *sU = lp_sm;                // [l][cs]  N * SX
    double *sX = sU + N * SX;          // [jj][cs] JT * SX
    double *sY = sX + LP_JT * SX;      // [jj][l]  JT * N
    // class-block source: table entries of the tile's rows (one per c) and K
    // indices (one per jj, s), the natural offset being r ks + k with
    // r = (o1 x_o1 + c xc) / ks and k = o2 x_o2 + j xj + s xs (host-checked)
    uint32_t *sRt = (uint32_t *)(sY + LP_JT * N);  // [c]      L
    uint32_t *sKt = sRt + LP_MAXL;                   // [jj][s]  JT * N
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int nw = (int)blockDim.x >> 6;
    for (int u = tid; u < (N + LP_JT) * SX; u += blockDim.x) lp_sm[u] = 0.0;
    __syncthreads();
    for (int u = tid; u < N * LN; u += blockDim.x) {
        const int cs = u % LN, l = u / LN, c = cs / N, s = cs - c * N;
        sU[l * SX + cs] = U[l * p.ul + s * p.us + c * p.uc];
    }
    const uint32_t o1 = blockIdx.x / p.n_o2, o2 = blockIdx.x % p.n_o2;
    const uint32_t xo = o1 * p.x_o1 + o2 * p.x_o2, oo = o1 * p.out_o1 + o2 * p.out_o2;
    lp_dbl4 eacc[LP_MAXB];
#pragma unroll
    for (int q = 0; q < LP_MAXB; ++q) eacc[q] = lp_dbl4{0.0, 0.0, 0.0, 0.0};
    // operand rows of this lane: l = lr (clamped; lanes with lr >= N supply zeros)
    const bool lok = lr < N;
    const int lrc = lok ? lr : N - 1;
    if (p.cls)
        for (int c = tid; c < L; c += blockDim.x) sRt[c] = p.rtab[(o1 * p.x_o1 + c * p.xc) / p.ks.d];
    // tile entries (jj, cs) of this thread: tid, tid + kT, ... walked
    // incrementally; every load of a stage is issued before the first LDS
    // store, so their latencies overlap (the stage is latency-bound)
    constexpr int XB = 8;
    constexpr int YIT = (LP_JT * N + kT - 1) / kT;
    const int nxit = (LP_JT * LN + kT - 1) / kT;  // entries per thread and tile
    const int jj0 = tid / LN, cs0 = tid - jj0 * LN, djj = kT / LN, dcs = kT - djj * LN;
    // class blocks selected without indexing the parameter arrays by a lane
    // value (which would read them from memory for every entry)
    const double *__restrict__ blk0 = p.blk[0], *__restrict__ blk1 = p.blk[1];
    const uint32_t ldb0 = p.ldb[0], ldb1 = p.ldb[1];
    for (uint32_t j0 = 0; j0 < p.NJ; j0 += LP_JT) {
        __syncthreads();  // previous tile consumed (and sU staged on the first pass)
        {   // Y tile and, for class blocks, the K table entries of the tile
            double yv[YIT];
            uint32_t kv[YIT];
#pragma unroll
            for (int it = 0; it < YIT; ++it) {
                const int idx = tid + it * kT, jj = idx / N, l = idx - jj * N;
                const uint32_t j = j0 + jj;
                const bool ok = idx < LP_JT * N && j < p.NJ;
                yv[it] = ok ? Y[oo + j * p.oj + l * p.ol] : 0.0;
                kv[it] = ok && p.cls ? p.ktab[o2 * p.x_o2 + j * p.xj + l * p.xs] : 0u;
            }
#pragma unroll
            for (int it = 0; it < YIT; ++it) {
                const int idx = tid + it * kT;
                if (idx < LP_JT * N) {
                    sY[idx] = yv[it];
                    sKt[idx] = kv[it];
                }
            }
        }
        if (p.cls) __syncthreads();
        {   // X tile, in batches of XB loads in flight per thread: every lane
            // loads (entries that are zero or outside the tile read U[0]
            // instead) and the selection happens at the LDS store, so no load
            // waits on a divergent branch
            int jj = jj0, cs = cs0;
            for (int it0 = 0; it0 < nxit; it0 += XB) {
                double xv[XB];
                uint32_t use = 0;
                int sj = jj, sc = cs;
#pragma unroll
                for (int it = 0; it < XB; ++it) {
                    const double *src = U;
                    const uint32_t j = j0 + jj;
                    if (jj < LP_JT && j < p.NJ) {
                        const int c = cs / N, s = cs - c * N;
                        if (p.cls) {
                            const uint32_t kt = sKt[jj * N + s], rt = sRt[c], b = kt >> 31;
                            if ((rt >> 31) == (b ^ p.zs)) {
                                src = (b ? blk1 : blk0) + ((size_t)(rt & ~Z2_PAR) * (b ? ldb1 : ldb0) +
                                                           (kt & ~Z2_PAR));
                                use |= 1u << it;
                            }
                        } else {
                            src = X + (xo + j * p.xj + c * p.xc + s * p.xs);
                            use |= 1u << it;
                        }
                    }
                    xv[it] = *src;
                    cs += dcs;
                    jj += djj;
                    if (cs >= LN) {
                        cs -= LN;
                        ++jj;
                    }
                }
#pragma unroll
                for (int it = 0; it < XB; ++it) {
                    if (sj < LP_JT) sX[sj * SX + sc] = (use >> it) & 1u ? xv[it] : 0.0;
                    sc += dcs;
                    sj += djj;
                    if (sc >= LN) {
                        sc -= LN;
                        ++sj;
                    }
                }
            }
        }
        __syncthreads();
        // outputs: one 16 j x 16 l block per wave (rows past NJ and columns
        // past N are computed from zeros and not stored)
        for (int jb = wave; jb < LP_JT / 16; jb += nw) {
            // two independent accumulation chains (k steps alternate)
            lp_dbl4 d = {0.0, 0.0, 0.0, 0.0}, d2 = {0.0, 0.0, 0.0, 0.0};
            const double *xa = sX + (jb * 16 + lr) * SX + lk;
            const double *ub = sU + lrc * SX + lk;
            int k0 = 0;
            for (; k0 + 8 <= KP; k0 += 8) {
                const double a0 = xa[k0], b0 = ub[k0], a1 = xa[k0 + 4], b1 = ub[k0 + 4];
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, lok ? b0 : 0.0, d, 0, 0, 0);
                d2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, lok ? b1 : 0.0, d2, 0, 0, 0);
            }
            if (k0 < KP) {
                const double a0 = xa[k0], b0 = ub[k0];
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, lok ? b0 : 0.0, d, 0, 0, 0);
            }
            d += d2;
            if (lok)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t j = j0 + jb * 16 + 4 * i + lk;
                    if (j < p.NJ) out[oo + j * p.oj + lr * p.ol] = d[i];
                }
        }
        // isometry adjoint: E blocks wave, wave + nw, ... (rows l, columns cs)
#pragma unroll
        for (int q = 0; q < LP_MAXB; ++q) {
            const int cb = wave + q * nw;
            if (cb >= NB) break;
            lp_dbl4 d = eacc[q];
            const int cc = cb * 16 + lr;  // column cs of this lane (>= LN: zeros)
            const int ccc = cc < LN ? cc : LN - 1;
#pragma unroll
            for (int k0 = 0; k0 < LP_JT; k0 += 4) {
                const double ya = sY[(k0 + lk) * N + lrc];
                const double xb = sX[(k0 + lk) * SX + ccc];
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(lok ? ya : 0.0, cc < LN ? xb : 0.0, d, 0, 0, 0);
            }
            eacc[q] = d;
        }
    }
    // row of `partial`: entry (l, s, c) at (l N + s) L + c
#pragma unroll
    for (int q = 0; q < LP_MAXB; ++q) {
        const int cb = wave + q * nw;
        if (cb >= NB) break;
        const int cs = cb * 16 + lr;
        if (cs >= LN) continue;
        const int c = cs / N, s = cs - c * N;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l = 4 * i + lk;
            if (l < N) partial[(size_t)blockIdx.x * (N * LN) + (l * N + s) * L + c] = eacc[q][i];
        }
    }
}

// Fixed-order reduction of the per-workgroup rows in two passes: group g of
// LP_G sums rows g, g + LP_G, ... into part2[g]; then part2 is summed in
// order and added into Ubar.
constexpr int LP_G = 64;
__global__ void __launch_bounds__(kT) lastprod_reduce1_kernel(const double *__restrict__ partial, uint32_t nblocks,
                                                              int nU, double *__restrict__ part2) {
    const int g = blockIdx.y;
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < nU; u += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (uint32_t b = g; b < nblocks; b += LP_G) acc += partial[(size_t)b * nU + u];
        part2[(size_t)g * nU + u] = acc;
    }
}

__global__ void __launch_bounds__(kT) lastprod_reduce2_kernel(LastProdParams p, const double *__restrict__ part2,
                                                              double *__restrict__ Ubar) {
    const int L = p.L, N = p.N, nU = N * N * L;
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < nU; u += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int g = 0; g < LP_G; ++g) acc += part2[(size_t)g * nU + u];
        const int c = u % L, s = (u / L) % N, l = u / (L * N);
        Ubar[l * p.ul + s * p.us + c * p.uc] += acc;
    }
}

template <int N>
void launch_lastprod_n(const LastProdParams &p, const double *X, const double *Y, const double *U, double *out,
                       double *Ubar, double *partial, hipStream_t s) {
    const uint32_t nb = p.n_o1 * p.n_o2;
    const size_t lds = sizeof(double) * ((size_t)(N + LP_JT) * lp_stride(p.L, N) + (size_t)LP_JT * N) +
                       sizeof(uint32_t) * ((size_t)LP_MAXL + (size_t)LP_JT * N);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)lastprod_adjoint_kernel<N>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    lastprod_adjoint_kernel<N><<<nb, kT, lds, s>>>(p, X, Y, U, out, partial);
    const int nU = N * N * p.L;
    double *part2 = partial + (size_t)nb * nU;  // LP_G rows after the per-workgroup ones
    const int gx = (nU + kT - 1) / kT;
    lastprod_reduce1_kernel<<<dim3(gx, LP_G), kT, 0, s>>>(partial, nb, nU, part2);
    lastprod_reduce2_kernel<<<gx, kT, 0, s>>>(p, part2, Ubar);
}

bool launch_lastprod_adjoint(const LastProdParams &p, const double *X, const double *Y, const double *U,
                             double *out, double *Ubar, double *partial, hipStream_t s) {
    if (p.L < 1 || p.L > LP_MAXL || p.N * p.N * p.L > kT * LP_UPT || p.n_o1 * p.n_o2 == 0) return false;
    switch (p.N) {
        case 2: launch_lastprod_n<2>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 3: launch_lastprod_n<3>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 4: launch_lastprod_n<4>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 5: launch_lastprod_n<5>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 6: launch_lastprod_n<6>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 7: launch_lastprod_n<7>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 8: launch_lastprod_n<8>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 9: launch_lastprod_n<9>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 10: launch_lastprod_n<10>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 11: launch_lastprod_n<11>(p, X, Y, U, out, Ubar, partial, s); return true;
        case 12: launch_lastprod_n<12>(p, X, Y, U, out, Ubar, partial, s); return true;
        default: return false;
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the truncated eigenvectors.  V: n x n row-major, column j is the
// j-th eigenvector (descending lam); U = V[:, :k]; Ubar: n x k row-major.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kT) eigh_adjoint_kernel(const double *__restrict__ V,
                                                          const double *__restrict__ lam,
                                                          const double *__restrict__ Ubar, int n, int k,
                                                          double *__restrict__ Ebar) {
    __shared__ double Ksh[169 * 13];  // (n - k) x k, n <= 169, k <= 13
    __shared__ double Zsh[169 * 13];  // n x k
    const int m = n - k;
    for (int idx = threadIdx.x; idx < m * k; idx += blockDim.x) {
        int j = idx / k, i = idx % k;
        double w = 0.0;
        for (int r = 0; r < n; ++r) w = fma(V[r * n + k + j], Ubar[r * k + i], w);
        Ksh[idx] = w / (lam[i] - lam[k + j]);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * k; idx += blockDim.x) {
        int r = idx / k, i = idx % k;
        double z = 0.0;
        for (int j = 0; j < m; ++j) z = fma(V[r * n + k + j], Ksh[j * k + i], z);
        Zsh[idx] = z;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        int r = idx / n, c = idx % n;
        double e1 = 0.0, e2 = 0.0;
        for (int i = 0; i < k; ++i) {
            e1 = fma(Zsh[r * k + i], V[c * n + i], e1);
            e2 = fma(Zsh[c * k + i], V[r * n + i], e2);
        }
        Ebar[idx] = 0.5 * (e1 + e2);
    }
}

void launch_eigh_adjoint(const double *V, const double *lam, const double *Ubar, int n, int k, double *Ebar,
                         hipStream_t s) {
    eigh_adjoint_kernel<<<1, kT, 0, s>>>(V, lam, Ubar, n, k, Ebar);
}

// ---------------------------------------------------------------------------
// Seed of the reverse pass: Tbar[x x y y z z t t] = value, zero elsewhere.
// ---------------------------------------------------------------------------
__global__ void diag_set_kernel(double *T, int D0, int D1, int D2, int D3, uint32_t s0, uint32_t s1, uint32_t s2,
                                uint32_t s3, double value) {
    uint32_t total = (uint32_t)D0 * D1 * D2 * D3;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        uint32_t r = e;
        uint32_t i3 = r % D3;
        r /= D3;
        uint32_t i2 = r % D2;
        r /= D2;
        uint32_t i1 = r % D1;
        uint32_t i0 = r / D1;
        T[i0 * s0 + i1 * s1 + i2 * s2 + i3 * s3] = value;
    }
}

void launch_diag_set(double *T, const int D[4], const uint32_t diag_st[4], double value, hipStream_t s) {
    diag_set_kernel<<<64, kT, 0, s>>>(T, D[0], D[1], D[2], D[3], diag_st[0], diag_st[1], diag_st[2], diag_st[3],
                                      value);
}

// ---------------------------------------------------------------------------
// <Tbar^(0), dT^(0)/dbeta> and <Tbar^(0), dT^(0)/dh> for the rank-8 tensor of
// bond dimension 2.  W[0] = (wc, ws), W[1][i] = (-1)^i W[0][i]; dW[0]/dbeta =
// (dwc, dws) with the same sign rule; v_up = e^{beta h}, v_dn = e^{-beta h}.
// out[0], out[1] get the two contractions divided by c0.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) site_dot_kernel(const double *__restrict__ Tbar, double wc, double ws,
                                                       double dwc, double dws, double beta, double h, double vu,
                                                       double vd, double inv_c0, double *__restrict__ out) {
    __shared__ double sb[256], sh[256];
    const int i = threadIdx.x;
    double m = 1.0, dm = 0.0;
    int odd = 0;
    for (int k = 0; k < 8; ++k) {
        const int b = (i >> (7 - k)) & 1;
        const double w = b ? ws : wc, dw = b ? dws : dwc;
        dm = dm * w + m * dw;
        m *= w;
        odd ^= b;
    }
    const double sg = odd ? -1.0 : 1.0;
    // T = vu m + vd sg m.  Written with the spin weights factored out: at
    // h = 0 (vu = vd = 1) dT/dh is then exactly 0 on the even entries (a
    // difference of two separately rounded products, which the compiler may
    // fuse into one FMA, would leave the rounding error of one of them)
    const double dT_dbeta = vu * (dm + h * m) + sg * vd * (dm - h * m);
    const double dT_dh = beta * m * (vu - sg * vd);
    sb[i] = Tbar[i] * dT_dbeta;
    sh[i] = Tbar[i] * dT_dh;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (i < w) {
            sb[i] += sb[i + w];
            sh[i] += sh[i + w];
        }
        __syncthreads();
    }
    if (i == 0) {
        out[0] = sb[0] * inv_c0;
        out[1] = sh[0] * inv_c0;
    }
}

void launch_site_dot(const double *Tbar, double wc, double ws, double dwc, double dws, double beta, double h,
                     double vu, double vd, double inv_c0, double *out, hipStream_t s) {
    site_dot_kernel<<<1, 256, 0, s>>>(Tbar, wc, ws, dwc, dws, beta, h, vu, vd, inv_c0, out);
}

}  // namespace hotrg
