// Memory-bound tensor kernels of one HOTRG step on gfx950: initial tensors,
// leg permutations, isometry (mode) products, norms, traces, Grams and the
// squeezed environments.  All FP64; every reduction runs in a fixed order so
// repeated runs are bitwise identical.
#include <utility>
#include "hotrg_internal.h"

namespace hotrg {

namespace {
constexpr int kThreads = 256;

inline int grid_for(size_t n, int per_block = kThreads, int cap = 65536) {
    size_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (size_t)cap) g = cap;
    return (int)g;
}
}  // namespace

// ---------------------------------------------------------------------------
// Initial tensors, Eqs. (2.2) and (2.6): entry i of the 2^8 array has leg k
// index (i >> (7 - k)) & 1; T = sum_s v_s prod_k W[s, i_k], S = sum_s s v_s ...
// ---------------------------------------------------------------------------
// W[1][i] = (-1)^i W[0][i] (W[1][0] = W[0][0], W[1][1] = -W[0][1]), so both
// spin states share one product chain of |W| and differ only by the sign
// (-1)^{#odd legs}: at h = 0 the Z2-odd entries of T (even of S) cancel
// exactly, with no contraction of a product into the final sum.
__global__ void init_site_kernel(double *T, double *S, double w00, double w01, double w10,
                                 double w11, double vu, double vd) {
    int i = threadIdx.x;
    double m = 1.0;
    int odd = 0;
    for (int k = 0; k < 8; ++k) {
        int b = (i >> (7 - k)) & 1;
        m *= b ? w01 : w00;
        odd ^= b;
    }
    (void)w10;
    (void)w11;
    const double pu = vu * m;
    const double pd = odd ? -(vd * m) : vd * m;
    T[i] = pu + pd;
    S[i] = pu - pd;
}

void launch_init_site(double *T, double *S, double w00, double w01, double w10, double w11,
                      double vu, double vd, hipStream_t s) {
    init_site_kernel<<<1, 256, 0, s>>>(T, S, w00, w01, w10, w11, vu, vd);
}

// ---------------------------------------------------------------------------
// Generic permutation / strided gather with a scale: out[o] = scale * in[map(o)].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) permute_kernel(PermParams p, const double *__restrict__ in,
                                                           double *__restrict__ out, double scale) {
    for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < p.total; o += gridDim.x * blockDim.x) {
        uint32_t rem = o, ib = 0;
        for (int k = p.nd - 1; k >= 0; --k) {
            uint32_t q = fast_div(rem, p.ext[k]);
            ib += (rem - q * p.ext[k].d) * p.in_st[k];
            rem = q;
        }
        out[o] = scale * in[ib];
    }
}

void launch_permute(const PermParams &p, const double *in, double *out, double scale, hipStream_t s) {
    if (p.total == 0) return;
    permute_kernel<<<grid_for(p.total), kThreads, 0, s>>>(p, in, out, scale);
}

// bf16 round-to-nearest-even of a float (finite inputs), raw bits.
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double bf16_value(uint16_t b) {
    return (double)__uint_as_float(((uint32_t)b) << 16);
}
// The same rounding (FP64 -> FP32 round-to-nearest-even, then FP32 -> bf16
// round-to-nearest-even) on gfx950's conversion instruction.  The empty asm
// keeps the compiler from fusing the two roundings into one FP64 -> bf16
// rounding (which differs from the bit form above in rare double-rounding
// cases).
__device__ __forceinline__ uint16_t bf16_bits_hw(double a) {
    float f = (float)a;
    asm volatile("" : "+v"(f));
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

// row-major operand offset -> packed GEMM layout (identity when not packed)
__device__ __forceinline__ size_t split_offset(const ExpandParams &p, uint32_t o) {
    if (!p.pack) return o;
    const uint32_t q = fast_div(o, p.pld);
    const uint32_t k = o - q * p.pld.d;
    const uint32_t r = q + p.prow0;
    return ((size_t)(r / PACK_ROWS) * p.pkb + k / PACK_K) * (PACK_ROWS * PACK_K) + (r % PACK_ROWS) * PACK_K +
           k % PACK_K;
}

template <bool SPLIT, bool RUN>
__global__ void __launch_bounds__(kThreads) iso_expand_kernel(ExpandParams p, const double *__restrict__ in,
                                                              const double *__restrict__ U,
                                                              double *__restrict__ out,
                                                              uint16_t *__restrict__ hi,
                                                              uint16_t *__restrict__ lo) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < p.threads; t += gridDim.x * blockDim.x) {
        uint32_t rem = t, ib = 0, ob = 0;
        for (int k = p.nd - 1; k >= 0; --k) {
            uint32_t q = fast_div(rem, p.ext[k]);
            uint32_t c = rem - q * p.ext[k].d;
            ib += c * p.in_st[k];
            ob += c * p.out_st[k];
            rem = q;
        }
        double v[XP_MAXS];
#pragma unroll
        for (int i = 0; i < XP_MAXS; ++i) v[i] = i < p.nsum ? in[ib + i * p.xs] : 0.0;
        for (int l1 = 0; l1 < p.L1; ++l1) {
            const double *Ul = U + l1 * p.u1;
            const uint32_t o = ob + l1 * p.o1;
            if (RUN) {
                // o2 == 1: a contiguous run of L2 outputs
                double r[XP_MAXS];
#pragma unroll
                for (int l2 = 0; l2 < XP_MAXS; ++l2) {
                    double acc = 0.0;
                    if (l2 < p.L2) {
#pragma unroll
                        for (int i = 0; i < XP_MAXS; ++i)
                            if (i < p.nsum) acc = fma(Ul[l2 * p.u2 + i * p.us], v[i], acc);
                    }
                    r[l2] = acc;
                }
                if (SPLIT) {
                    // two consecutive outputs starting at an even offset are
                    // adjacent in both layouts (row lengths are even), so they
                    // go out as one 4-byte store per array
                    bool done = false;
#pragma unroll
                    for (int l2 = 0; l2 < XP_MAXS; ++l2) {
                        if (l2 >= p.L2) break;
                        if (done) {
                            done = false;
                            continue;
                        }
                        const uint16_t h = bf16_bits((float)r[l2]);
                        const uint16_t lw = bf16_bits((float)(r[l2] - bf16_value(h)));
                        const size_t po = split_offset(p, o + l2);
                        if (((o + l2) & 1) == 0 && l2 + 1 < p.L2 && l2 + 1 < XP_MAXS) {
                            const uint16_t h2 = bf16_bits((float)r[l2 + 1]);
                            const uint16_t lw2 = bf16_bits((float)(r[l2 + 1] - bf16_value(h2)));
                            *(uint32_t *)(hi + po) = (uint32_t)h | ((uint32_t)h2 << 16);
                            *(uint32_t *)(lo + po) = (uint32_t)lw | ((uint32_t)lw2 << 16);
                            done = true;
                        } else {
                            hi[po] = h;
                            lo[po] = lw;
                        }
                    }
                } else {
#pragma unroll
                    for (int l2 = 0; l2 < XP_MAXS; ++l2) {
                        if (l2 >= p.L2) break;
                        out[o + l2] = r[l2];
                    }
                }
            } else {
                for (int l2 = 0; l2 < p.L2; ++l2) {
                    double acc = 0.0;
#pragma unroll
                    for (int i = 0; i < XP_MAXS; ++i)
                        if (i < p.nsum) acc = fma(Ul[l2 * p.u2 + i * p.us], v[i], acc);
                    const uint32_t oo = o + l2 * p.o2;
                    if (SPLIT) {
                        uint16_t h = bf16_bits((float)acc);
                        const size_t po = split_offset(p, oo);
                        hi[po] = h;
                        lo[po] = bf16_bits((float)(acc - bf16_value(h)));
                    } else {
                        out[oo] = acc;
                    }
                }
            }
        }
    }
}

// Specialisation for the shapes of the HOTRG step, where the summed index and
// the second loop index run over the same leg dimension N (nsum == L2 == N):
// the block first stages the isometry block U[l1, l2, i] (in use order) in
// LDS, so that the fully unrolled inner loop reads it with wave-uniform LDS
// loads instead of one dependent scalar load per FMA.  Same arithmetic, in
// the same order, as iso_expand_kernel.
template <bool SPLIT, bool RUN, int N>
__global__ void __launch_bounds__(kThreads) iso_expand_lds_kernel(ExpandParams p, const double *__restrict__ in,
                                                                  const double *__restrict__ U,
                                                                  double *__restrict__ out,
                                                                  uint16_t *__restrict__ hi,
                                                                  uint16_t *__restrict__ lo) {
    extern __shared__ double sU[];  // [L1][N][N]
    const int nU = p.L1 * N * N;
    for (int idx = threadIdx.x; idx < nU; idx += blockDim.x) {
        const int i = idx % N, l2 = (idx / N) % N, l1 = idx / (N * N);
        sU[idx] = U[l1 * p.u1 + l2 * p.u2 + i * p.us];
    }
    __syncthreads();
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < p.threads; t += gridDim.x * blockDim.x) {
        uint32_t rem = t, ib = 0, ob = 0;
        for (int k = p.nd - 1; k >= 0; --k) {
            uint32_t q = fast_div(rem, p.ext[k]);
            uint32_t c = rem - q * p.ext[k].d;
            ib += c * p.in_st[k];
            ob += c * p.out_st[k];
            rem = q;
        }
        double v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = in[ib + i * p.xs];
        for (int l1 = 0; l1 < p.L1; ++l1) {
            const double *ul = sU + l1 * N * N;
            const uint32_t o = ob + l1 * p.o1;
            // outputs in pairs (l2, l2 + 1): few live registers; a pair that
            // starts at an even offset of a contiguous run is adjacent in both
            // layouts (row lengths are even) and goes out as 4-byte stores
#pragma unroll 1
            for (int l2 = 0; l2 < N; l2 += 2) {
                const bool two = l2 + 1 < N;
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    a0 = fma(ul[l2 * N + i], v[i], a0);
                    if (two) a1 = fma(ul[(l2 + 1) * N + i], v[i], a1);
                }
                const uint32_t o0 = RUN ? o + l2 : o + l2 * p.o2;
                const uint32_t o1 = RUN ? o0 + 1 : o0 + p.o2;
                if (SPLIT) {
                    const uint16_t h0 = bf16_bits((float)a0), w0 = bf16_bits((float)(a0 - bf16_value(h0)));
                    const size_t p0 = split_offset(p, o0);
                    if (two) {
                        const uint16_t h1 = bf16_bits((float)a1), w1 = bf16_bits((float)(a1 - bf16_value(h1)));
                        if (RUN && (o0 & 1) == 0) {
                            *(uint32_t *)(hi + p0) = (uint32_t)h0 | ((uint32_t)h1 << 16);
                            *(uint32_t *)(lo + p0) = (uint32_t)w0 | ((uint32_t)w1 << 16);
                        } else {
                            const size_t p1 = split_offset(p, o1);
                            hi[p0] = h0;
                            lo[p0] = w0;
                            hi[p1] = h1;
                            lo[p1] = w1;
                        }
                    } else {
                        hi[p0] = h0;
                        lo[p0] = w0;
                    }
                } else {
                    out[o0] = a0;
                    if (two) out[o1] = a1;
                }
            }
        }
    }
}

// Z2 block scatter of the last isometry product (see ExpandParams): the
// destination of every output is looked up first, outputs that the parity
// structure makes exactly zero are neither computed nor written, and the rest
// go to their parity block (FP64 row-major, or bf16 hi / lo in the packed
// layout).  Same arithmetic, in the same order, as iso_expand_lds_kernel.
template <bool SPLIT, int N>
__global__ void __launch_bounds__(kThreads) iso_expand_z2_kernel(ExpandParams p, const double *__restrict__ in,
                                                                 const double *__restrict__ U) {
    extern __shared__ double sZ[];  // [L1][N][N]
    const int nU = p.L1 * N * N;
    for (int idx = threadIdx.x; idx < nU; idx += blockDim.x) {
        const int i = idx % N, l2 = (idx / N) % N, l1 = idx / (N * N);
        sZ[idx] = U[l1 * p.u1 + l2 * p.u2 + i * p.us];
    }
    __syncthreads();
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < p.threads; t += gridDim.x * blockDim.x) {
        uint32_t rem = t, ib = 0, ob = 0;
        for (int k = p.nd - 1; k >= 0; --k) {
            uint32_t q = fast_div(rem, p.ext[k]);
            uint32_t c = rem - q * p.ext[k].d;
            ib += c * p.in_st[k];
            ob += c * p.out_st[k];
            rem = q;
        }
        double v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = in[ib + i * p.xs];
        for (int l1 = 0; l1 < p.L1; ++l1) {
            const double *ul = sZ + l1 * N * N;
            const uint32_t o = ob + l1 * p.o1;
#pragma unroll 1
            for (int l2 = 0; l2 < N; ++l2) {
                const uint32_t oo = o + l2 * p.o2;
                const uint32_t r = fast_div(oo, p.zld);
                const uint32_t k = oo - r * p.zld.d;
                const uint32_t rt = p.rtab[r], kt = p.ktab[k];
                const uint32_t blk = kt >> 31, g = blk ^ p.zs;
                if ((rt >> 31) != (p.zP ^ g)) continue;  // structurally zero
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < N; ++i) acc = fma(ul[l2 * N + i], v[i], acc);
                const uint32_t row = p.zrow_off[g] + (rt & ~Z2_PAR), col = kt & ~Z2_PAR;
                if (SPLIT) {
                    const uint16_t h = bf16_bits((float)acc);
                    const size_t po = ((size_t)(row / PACK_ROWS) * p.zpkb[blk] + col / PACK_K) * (PACK_ROWS * PACK_K) +
                                      (row % PACK_ROWS) * PACK_K + col % PACK_K;
                    p.zhi[blk][po] = h;
                    p.zlo[blk][po] = bf16_bits((float)(acc - bf16_value(h)));
                } else {
                    p.zout[blk][(size_t)row * p.zld_out[blk] + col] = acc;
                }
            }
        }
    }
}

// Run form of the Z2 scatter (z2 == 2): a thread splits its base offset
// into (row, K) once, loads the class entries of its N outputs along the
// second loop once, and per step of the first loop looks up one row: the row
// decides the only block that can receive outputs (block = row parity ^ zP ^
// zs), and the outputs whose K class is that block are computed and stored.
template <bool SPLIT, int N>
__global__ void __launch_bounds__(kThreads) iso_expand_z2run_kernel(ExpandParams p, const double *__restrict__ in,
                                                                    const double *__restrict__ U) {
    extern __shared__ double sZ[];  // [L1][N][N]
    const int nU = p.L1 * N * N;
    for (int idx = threadIdx.x; idx < nU; idx += blockDim.x) {
        const int i = idx % N, l2 = (idx / N) % N, l1 = idx / (N * N);
        sZ[idx] = U[l1 * p.u1 + l2 * p.u2 + i * p.us];
    }
    __syncthreads();
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < p.threads; t += gridDim.x * blockDim.x) {
        uint32_t rem = t, ib = 0, ob = 0;
        for (int k = p.nd - 1; k >= 0; --k) {
            uint32_t q = fast_div(rem, p.ext[k]);
            uint32_t c = rem - q * p.ext[k].d;
            ib += c * p.in_st[k];
            ob += c * p.out_st[k];
            rem = q;
        }
        const uint32_t r0 = fast_div(ob, p.zld);
        const uint32_t k0 = ob - r0 * p.zld.d;
        uint32_t kt[N];
#pragma unroll
        for (int l2 = 0; l2 < N; ++l2) kt[l2] = p.ktab[k0 + l2 * p.o2];
        double v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = in[ib + i * p.xs];
        for (int l1 = 0; l1 < p.L1; ++l1) {
            const uint32_t rt = p.rtab[r0 + l1 * p.zrs];
            const uint32_t blk = (rt >> 31) ^ p.zP ^ p.zs, g = blk ^ p.zs;
            const uint32_t row = p.zrow_off[g] + (rt & ~Z2_PAR);
            const double *ul = sZ + l1 * N * N;
            const size_t rbase = SPLIT ? (size_t)(row / PACK_ROWS) * p.zpkb[blk] * (PACK_ROWS * PACK_K) +
                                             (row % PACK_ROWS) * PACK_K
                                       : (size_t)row * p.zld_out[blk];
            uint16_t *hi = SPLIT ? p.zhi[blk] : nullptr;
            uint16_t *lo = SPLIT ? p.zlo[blk] : nullptr;
            double *out = SPLIT ? nullptr : p.zout[blk];
            // bf16: an output at an even column whose successor in the run is
            // the next column goes out with it as one 4-byte (hi, hi') and one
            // (lo, lo') store (both in one 32-k piece of the packed row)
            bool held = false;
            uint32_t hcol = 0;
            uint16_t hh = 0, hl = 0;
#pragma unroll
            for (int l2 = 0; l2 < N; ++l2) {
                if ((kt[l2] >> 31) != blk) continue;  // structurally zero
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < N; ++i) acc = fma(ul[l2 * N + i], v[i], acc);
                const uint32_t col = kt[l2] & ~Z2_PAR;
                if (SPLIT) {
                    const uint16_t h = bf16_bits((float)acc);
                    const uint16_t l = bf16_bits((float)(acc - bf16_value(h)));
                    if (held && col == hcol + 1) {
                        const size_t po = rbase + (size_t)(hcol / PACK_K) * (PACK_ROWS * PACK_K) + hcol % PACK_K;
                        *(uint32_t *)(hi + po) = (uint32_t)hh | ((uint32_t)h << 16);
                        *(uint32_t *)(lo + po) = (uint32_t)hl | ((uint32_t)l << 16);
                        held = false;
                        continue;
                    }
                    if (held) {
                        const size_t po = rbase + (size_t)(hcol / PACK_K) * (PACK_ROWS * PACK_K) + hcol % PACK_K;
                        hi[po] = hh;
                        lo[po] = hl;
                        held = false;
                    }
                    if ((col & 1) == 0 && p.zpair) {
                        held = true;
                        hcol = col;
                        hh = h;
                        hl = l;
                    } else {
                        const size_t po = rbase + (size_t)(col / PACK_K) * (PACK_ROWS * PACK_K) + col % PACK_K;
                        hi[po] = h;
                        lo[po] = l;
                    }
                } else {
                    out[rbase + col] = acc;
                }
            }
            if (SPLIT && held) {
                const size_t po = rbase + (size_t)(hcol / PACK_K) * (PACK_ROWS * PACK_K) + hcol % PACK_K;
                hi[po] = hh;
                lo[po] = hl;
            }
        }
    }
}

// Tile form of the Z2 scatter (z2 == 3, bf16 hi / lo only; the layout of the
// thread dims is described at ExpandParams).  Each tile is a rectangle of
// natural rows [R0, R1) x natural K indices [K0, K1): in class order its
// outputs form, per block, the class rows of one parity in a contiguous range
// times the class-b K positions in a contiguous range.  The tile's threads
// compute the allowed outputs with the arithmetic of iso_expand_z2run_kernel
// and put them into an LDS copy of those two rectangles; the rectangles then
// go out in the packed layout as 16-byte pieces (8 k of one row), lanes
// ordered so that consecutive rows of one 32-k piece (consecutive 64-byte
// runs) are written together.  Only the pieces at the two K ends of a
// rectangle, shared with the neighbouring K groups, are written element by
// element.
//
// Thread slots: a unit's inner threads are listed by the parity of their K
// run (tperm, each parity padded to whole waves with idle slots ~0u), so in
// every wave the test "K class of loop index l2 == block of row l1" has one
// answer for all lanes and the skipped outputs cost no issue slots.
//
// Isometry zeros: a column of the isometry lies in one parity sector, so for
// an output (l1, l2) only the summed indices i of parity need(l1, l2) =
// lab1(l1) ^ lab2(l2) contribute (the others meet exact zeros).  For the
// outputs a wave computes at one l1 that parity is the same for every lane.
// The input run is loaded twice, compacted to the indices of parity 0 (v0)
// and of parity 1 (v1), NH values each (zero-padded), and tU holds the
// isometry block as [l1][l2][j], j < NH, with entry j the j-th index of
// parity need(l1, l2) (zero past the count): NH FMAs per output instead of N,
// in the same order over the contributing indices (the dropped terms are
// exact zeros).  tU is read with wave-uniform addresses (scalar loads).
//
// The next tile's input runs and K table entries are loaded before the
// current tile's LDS rectangles are written out.
template <int N, int NH>
__global__ void __launch_bounds__(Z2TILE_MAX_THREADS) iso_expand_z2tile_kernel(ExpandParams p,
                                                                              const double *__restrict__ in,
                                                                              const double *__restrict__ tU) {
    extern __shared__ __align__(16) uint16_t sZt[];
    uint16_t *th = sZt;
    uint16_t *tl = th + (size_t)p.tupb * p.L1 * p.tLD;
    const uint32_t LD = p.tLD;
    const uint32_t per_group = (p.tNRP + p.tupb - 1) / p.tupb;
    const uint32_t ntiles = p.tKg * per_group;
    const uint32_t unit = threadIdx.x / p.tslots, slot = threadIdx.x - unit * p.tslots;
    const uint32_t inner = p.tperm[slot];
    // natural output offset and input offset of thread t of the launch
    auto offsets = [&](uint32_t t, uint32_t &ib, uint32_t &ob) {
        uint32_t rem = t;
        ib = 0;
        ob = 0;
        for (int k = p.nd - 1; k >= 0; --k) {
            const uint32_t q = fast_div(rem, p.ext[k]);
            const uint32_t c = rem - q * p.ext[k].d;
            ib += c * p.in_st[k];
            ob += c * p.out_st[k];
            rem = q;
        }
    };
    // entries of class b before natural K index k (rows: of parity q before row r)
    auto kcount = [&](uint32_t k, uint32_t b) -> uint32_t {
        if (k >= p.zKc[0] + p.zKc[1]) return p.zKc[b];
        const uint32_t kt = p.ktab[k], pos = kt & ~Z2_PAR;
        return (kt >> 31) == b ? pos : k - pos;
    };
    auto rcount = [&](uint32_t r, uint32_t q) -> uint32_t {
        if (r >= p.zM) return p.zNr[q];
        const uint32_t rt = p.rtab[r], pos = rt & ~Z2_PAR;
        return (rt >> 31) == q ? pos : r - pos;
    };
    // this thread's work in a tile: input runs and K table entries
    double v0[NH], v1[NH];
    uint32_t kt[N];
    uint32_t r0 = 0;
    auto fetch = [&](uint32_t tl_) -> bool {
        const uint32_t kg = tl_ / per_group, u0 = (tl_ - kg * per_group) * p.tupb;
        if (unit >= min(p.tupb, p.tNRP - u0) || inner == ~0u) return false;
        uint32_t ib, ob;
        offsets((kg * p.tNRP + u0) * p.tP + unit * p.tP + inner, ib, ob);
        r0 = fast_div(ob, p.zld);
        const uint32_t k0 = ob - r0 * p.zld.d;
#pragma unroll
        for (int l2 = 0; l2 < N; ++l2) kt[l2] = p.ktab[k0 + l2 * p.o2];
#pragma unroll
        for (int j = 0; j < NH; ++j) {
            const uint32_t i0 = (uint32_t)(p.tI[0] >> (4 * j)) & 15u, i1 = (uint32_t)(p.tI[1] >> (4 * j)) & 15u;
            v0[j] = j < (int)p.tnI[0] ? in[ib + i0 * p.xs] : 0.0;
            v1[j] = j < (int)p.tnI[1] ? in[ib + i1 * p.xs] : 0.0;
        }
        return true;
    };
    uint32_t tile = blockIdx.x;
    bool active = tile < ntiles && fetch(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const uint32_t kg = tile / per_group, u0 = (tile - kg * per_group) * p.tupb;
        const uint32_t nu = min(p.tupb, p.tNRP - u0);
        uint32_t ib0, ob0;
        offsets((kg * p.tNRP + u0) * p.tP, ib0, ob0);
        const uint32_t R0 = fast_div(ob0, p.zld), K0 = ob0 - R0 * p.zld.d;
        const uint32_t R1 = R0 + nu * p.L1, K1 = K0 + p.tnK;
        // per block b: class rows [rb0, rb0 + nr) of parity zP ^ zs ^ b (LDS
        // rows from lr0), class K positions [ck, ck + nk) (LDS columns from the
        // 8-aligned cal)
        uint32_t nr[2], rb0[2], lr0[2], ck[2], nk[2], cal[2];
#pragma unroll
        for (uint32_t b = 0; b < 2; ++b) {
            const uint32_t q = b ^ p.zP ^ p.zs;
            rb0[b] = rcount(R0, q);
            nr[b] = rcount(R1, q) - rb0[b];
            ck[b] = kcount(K0, b);
            nk[b] = kcount(K1, b) - ck[b];
            cal[b] = ck[b] & ~7u;
        }
        lr0[0] = 0;
        lr0[1] = nr[0];
        if (active) {
            // class of loop index l2 = Q ^ lab2(l2)
            const uint32_t Q = (kt[0] >> 31) ^ (p.tlab2 & 1u);
            for (int l1 = 0; l1 < p.L1; ++l1) {
                const uint32_t rt = p.rtab[r0 + l1];
                const uint32_t blk = (rt >> 31) ^ p.zP ^ p.zs;
                // LDS index of class column col: lbase + col (col >= cal[blk])
                const uint32_t lbase = (lr0[blk] + (rt & ~Z2_PAR) - rb0[blk]) * LD - cal[blk];
                const double *ul = tU + (size_t)l1 * N * NH;
                auto row = [&](const double (&w)[NH]) {
#pragma unroll
                    for (int l2 = 0; l2 < N; ++l2) {
                        if ((kt[l2] >> 31) != blk) continue;  // structurally zero
                        double acc = 0.0;
#pragma unroll
                        for (int j = 0; j < NH; ++j) acc = fma(ul[l2 * NH + j], w[j], acc);
                        const uint16_t h = bf16_bits_hw(acc);
                        const uint32_t col = kt[l2] & ~Z2_PAR;
                        th[lbase + col] = h;
                        tl[lbase + col] = bf16_bits_hw(acc - bf16_value(h));
                    }
                };
                // parity of the contributing summed indices (the allowed l2 have lab2 = Q ^ blk)
                if ((((p.tlab1 >> l1) & 1u) ^ Q ^ blk) != 0u)
                    row(v1);
                else
                    row(v0);
            }
        }
        // the next tile's loads go out before this tile's rectangles
        const uint32_t next = tile + gridDim.x;
        const uint32_t rb0c[2] = {rb0[0], rb0[1]};
        active = next < ntiles && fetch(next);
        __syncthreads();
#pragma unroll
        for (uint32_t b = 0; b < 2; ++b) {
            if (nr[b] == 0 || nk[b] == 0) continue;
            const uint32_t g = b ^ p.zs;
            const uint32_t prow0 = p.zrow_off[g] + rb0c[b];
            const uint32_t j0 = ck[b] >> 5, np = ((ck[b] + nk[b] - 1) >> 5) - j0 + 1;
            const uint32_t items = np * nr[b] * 4, kend = ck[b] + nk[b];
            uint16_t *__restrict__ ghi = p.zhi[b];
            uint16_t *__restrict__ glo = p.zlo[b];
            for (uint32_t w = threadIdx.x; w < items; w += blockDim.x) {
                const uint32_t q = w & 3, rw = w >> 2;
                const uint32_t jj = rw / nr[b], r = rw - jj * nr[b];
                const uint32_t c0 = (j0 + jj) * 32 + q * 8;
                if (c0 + 8 <= ck[b] || c0 >= kend) continue;
                const uint32_t prow = prow0 + r;
                const size_t go = ((size_t)(prow / PACK_ROWS) * p.zpkb[b] + (j0 + jj)) * (PACK_ROWS * PACK_K) +
                                  (prow % PACK_ROWS) * PACK_K + q * 8;
                const uint32_t lo_ = (lr0[b] + r) * LD + (c0 - cal[b]);
                if (c0 >= ck[b] && c0 + 8 <= kend) {
                    *(uint4 *)(ghi + go) = *(const uint4 *)(th + lo_);
                    *(uint4 *)(glo + go) = *(const uint4 *)(tl + lo_);
                } else {
#pragma unroll
                    for (uint32_t e = 0; e < 8; ++e)
                        if (c0 + e >= ck[b] && c0 + e < kend) {
                            ghi[go + e] = th[lo_ + e];
                            glo[go + e] = tl[lo_ + e];
                        }
                }
            }
        }
        __syncthreads();
    }
}

// Transposed Z2 block scatter of the reverse pass (z2 == 4): the natural
// offset o = K zld + r of a transposed operand slice (rows = inner K indices,
// columns = GEMM rows r) is split into (K, r); the thread's first loop steps
// r by o1 (< zld), the second steps K by o2 / zld.  An output with K class b
// goes to block b (GEMM class g = b ^ zs) and is structurally zero unless the
// parity of r is zP ^ g; block b gets row = K position, column = zrow_off[g] +
// r position (FP64 row-major with row length zld_out[b], or bf16 hi / lo in the
// packed layout with zpkb[b] = zld_out[b] / 32).  Same arithmetic as
// iso_expand_kernel.
template <bool SPLIT, int N>
__global__ void __launch_bounds__(kThreads) iso_expand_z2t_kernel(ExpandParams p, const double *__restrict__ in,
                                                                  const double *__restrict__ U) {
    extern __shared__ double sZ[];  // [L1][N][N]
    const int nU = p.L1 * N * N;
    for (int idx = threadIdx.x; idx < nU; idx += blockDim.x) {
        const int i = idx % N, l2 = (idx / N) % N, l1 = idx / (N * N);
        sZ[idx] = U[l1 * p.u1 + l2 * p.u2 + i * p.us];
    }
    __syncthreads();
    const uint32_t kstep = p.zrs;  // K step of the second loop
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < p.threads; t += gridDim.x * blockDim.x) {
        uint32_t rem = t, ib = 0, ob = 0;
        for (int k = p.nd - 1; k >= 0; --k) {
            uint32_t q = fast_div(rem, p.ext[k]);
            uint32_t c = rem - q * p.ext[k].d;
            ib += c * p.in_st[k];
            ob += c * p.out_st[k];
            rem = q;
        }
        const uint32_t K0 = fast_div(ob, p.zld);
        const uint32_t r0 = ob - K0 * p.zld.d;
        uint32_t kt[N];
#pragma unroll
        for (int l2 = 0; l2 < N; ++l2) kt[l2] = p.ktab[K0 + l2 * kstep];
        double v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = in[ib + i * p.xs];
        for (int l1 = 0; l1 < p.L1; ++l1) {
            const uint32_t rt = p.rtab[r0 + l1 * p.o1];
            const double *ul = sZ + l1 * N * N;
#pragma unroll
            for (int l2 = 0; l2 < N; ++l2) {
                const uint32_t blk = kt[l2] >> 31, g = blk ^ p.zs;
                if ((rt >> 31) != (p.zP ^ g)) continue;  // structurally zero
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < N; ++i) acc = fma(ul[l2 * N + i], v[i], acc);
                const uint32_t row = kt[l2] & ~Z2_PAR, col = p.zrow_off[g] + (rt & ~Z2_PAR);
                if (SPLIT) {
                    const uint16_t h = bf16_bits((float)acc);
                    const size_t po = ((size_t)(row / PACK_ROWS) * p.zpkb[blk] + col / PACK_K) * (PACK_ROWS * PACK_K) +
                                      (row % PACK_ROWS) * PACK_K + col % PACK_K;
                    p.zhi[blk][po] = h;
                    p.zlo[blk][po] = bf16_bits((float)(acc - bf16_value(h)));
                } else {
                    p.zout[blk][(size_t)row * p.zld_out[blk] + col] = acc;
                }
            }
        }
    }
}

template <int N>
void launch_iso_expand_z2t(const ExpandParams &p, bool split, const double *in, const double *U, hipStream_t s) {
    const size_t lds = (size_t)p.L1 * N * N * sizeof(double);
    const int g = grid_for(p.threads, kThreads, 4096);
    if (split) iso_expand_z2t_kernel<true, N><<<g, kThreads, lds, s>>>(p, in, U);
    else iso_expand_z2t_kernel<false, N><<<g, kThreads, lds, s>>>(p, in, U);
}

// C_bar in class blocks (reverse pass, pure T): for class g, rows and columns
// are the natural GEMM rows of parity g (inv lists them in class order);
// C_g[i][j] = scale * Tbar[roff[inv_g[i]] + coff[inv_g[j]]], and its transpose.
__global__ void __launch_bounds__(kThreads) z2_cbar_kernel(const double *__restrict__ Tbar,
                                                          const uint32_t *__restrict__ inv,
                                                          const uint32_t *__restrict__ roff,
                                                          const uint32_t *__restrict__ coff, uint32_t N0,
                                                          FastDiv n0, FastDiv n1, double scale,
                                                          double *__restrict__ Cg, double *__restrict__ CgT) {
    const uint32_t N1 = n1.d, tot0 = N0 * N0, tot = tot0 + N1 * N1;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
        const bool g1 = e >= tot0;
        const uint32_t loc = g1 ? e - tot0 : e;
        const FastDiv &nd = g1 ? n1 : n0;
        const uint32_t i = fast_div(loc, nd), j = loc - i * nd.d;
        const uint32_t *iv = inv + (g1 ? N0 : 0);
        const double v = scale * Tbar[roff[iv[i]] + coff[iv[j]]];
        const size_t base = g1 ? tot0 : 0;
        Cg[base + (size_t)i * nd.d + j] = v;
        CgT[base + (size_t)j * nd.d + i] = v;
    }
}

void launch_z2_cbar(const double *Tbar, const uint32_t *inv, const uint32_t *roff, const uint32_t *coff,
                    uint32_t N0, uint32_t N1, double scale, double *Cg, double *CgT, hipStream_t s) {
    const size_t tot = (size_t)N0 * N0 + (size_t)N1 * N1;
    if (tot == 0) return;
    z2_cbar_kernel<<<grid_for(tot), kThreads, 0, s>>>(Tbar, inv, roff, coff, N0, make_fastdiv(N0 ? N0 : 1),
                                                      make_fastdiv(N1 ? N1 : 1), scale, Cg, CgT);
}

// Class-block GEMM outputs -> natural [R][Ks] operand adjoint (reverse pass):
// out[r][K] = blk_b[pos(r) * ldb[b] + pos(K)] when the parity of r is
// zP ^ b ^ zs (b the class of K), else exactly 0.
__global__ void __launch_bounds__(kThreads) z2_unscatter_kernel(const double *__restrict__ b0,
                                                               const double *__restrict__ b1, uint32_t ld0,
                                                               uint32_t ld1, const uint32_t *__restrict__ rtab,
                                                               const uint32_t *__restrict__ ktab, uint32_t zs,
                                                               uint32_t zP, FastDiv ks, uint32_t R,
                                                               double *__restrict__ out) {
    const size_t tot = (size_t)R * ks.d;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
        const uint32_t r = fast_div(e, ks), k = e - r * ks.d;
        const uint32_t kt = ktab[k], rt = rtab[r];
        const uint32_t b = kt >> 31;
        double v = 0.0;
        if ((rt >> 31) == (zP ^ b ^ zs))
            v = b ? b1[(size_t)(rt & ~Z2_PAR) * ld1 + (kt & ~Z2_PAR)] : b0[(size_t)(rt & ~Z2_PAR) * ld0 + (kt & ~Z2_PAR)];
        out[e] = v;
    }
}

void launch_z2_unscatter(const double *b0, const double *b1, uint32_t ld0, uint32_t ld1, const uint32_t *rtab,
                         const uint32_t *ktab, uint32_t zs, uint32_t zP, uint32_t Ks, uint32_t R, double *out,
                         hipStream_t s) {
    const size_t tot = (size_t)R * Ks;
    if (tot == 0) return;
    z2_unscatter_kernel<<<grid_for(tot), kThreads, 0, s>>>(b0, b1, ld0, ld1, rtab, ktab, zs, zP, make_fastdiv(Ks), R,
                                                           out);
}

// tU[j] = src[idx[j]] (0 where idx[j] < 0)
__global__ void gather_or_zero_kernel(const double *__restrict__ src, const int32_t *__restrict__ idx,
                                      double *__restrict__ dst, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) dst[j] = idx[j] >= 0 ? src[idx[j]] : 0.0;
}
void launch_gather_or_zero(const double *src, const int32_t *idx, double *dst, int n, hipStream_t s) {
    if (n > 0) gather_or_zero_kernel<<<(n + 255) / 256, 256, 0, s>>>(src, idx, dst, n);
}

template <int N, int NH>
void launch_z2tile(const ExpandParams &p, const double *in, hipStream_t s) {
    const uint32_t per_group = (p.tNRP + p.tupb - 1) / p.tupb;
    const size_t tiles = (size_t)p.tKg * per_group;
    const int g = (int)(tiles < 8192 ? tiles : 8192);
    iso_expand_z2tile_kernel<N, NH><<<g, (int)(p.tupb * p.tslots), z2tile_lds_bytes(p), s>>>(p, in, p.tU);
}

// NH = N always; for N >= 8 also the two near-even splits
template <int N>
void launch_z2tile_nh(const ExpandParams &p, const double *in, hipStream_t s) {
    constexpr int H = (N + 1) / 2;
    if constexpr (N >= 8) {
        if (p.tNH == H) return launch_z2tile<N, H>(p, in, s);
        if (p.tNH == H + 1) return launch_z2tile<N, H + 1>(p, in, s);
    }
    launch_z2tile<N, N>(p, in, s);
}

int z2tile_nh(int N, int nmax) {
    const int H = (N + 1) / 2;
    return N >= 8 && nmax <= H ? H : (N >= 8 && nmax == H + 1 ? H + 1 : N);
}

template <int N>
void launch_iso_expand_z2(const ExpandParams &p, bool split, const double *in, const double *U, hipStream_t s) {
    if (p.z2 == 3) {
        // the host checked the tile layout, split, the slot table, the thread
        // count and the LDS size, and wrote tU
        launch_z2tile_nh<N>(p, in, s);
        return;
    }
    const size_t lds = (size_t)p.L1 * N * N * sizeof(double);
    const int g = grid_for(p.threads, kThreads, 4096);
    if (p.z2 == 2) {
        if (split) iso_expand_z2run_kernel<true, N><<<g, kThreads, lds, s>>>(p, in, U);
        else iso_expand_z2run_kernel<false, N><<<g, kThreads, lds, s>>>(p, in, U);
        return;
    }
    if (split) iso_expand_z2_kernel<true, N><<<g, kThreads, lds, s>>>(p, in, U);
    else iso_expand_z2_kernel<false, N><<<g, kThreads, lds, s>>>(p, in, U);
}

template <int N>
void launch_iso_expand_lds(const ExpandParams &p, const double *in, const double *U, double *out, uint16_t *hi,
                           uint16_t *lo, hipStream_t s) {
    const size_t lds = (size_t)p.L1 * N * N * sizeof(double);
    const int g = grid_for(p.threads, kThreads, 4096);  // blocks loop, so U is staged only 4096 times
    const bool run = p.o2 == 1;
    if (hi) {
        if (run) iso_expand_lds_kernel<true, true, N><<<g, kThreads, lds, s>>>(p, in, U, out, hi, lo);
        else iso_expand_lds_kernel<true, false, N><<<g, kThreads, lds, s>>>(p, in, U, out, hi, lo);
    } else {
        if (run) iso_expand_lds_kernel<false, true, N><<<g, kThreads, lds, s>>>(p, in, U, out, hi, lo);
        else iso_expand_lds_kernel<false, false, N><<<g, kThreads, lds, s>>>(p, in, U, out, hi, lo);
    }
}

// bf16 hi/lo outputs written as 4-byte (hi, hi') / (lo, lo') pairs of adjacent
// outputs, laid out so that consecutive lanes write consecutive pairs.
// PAIR_RUN (the l2 loop is an output run, o2 == 1): unit u = t * N/2 + m
//   computes outputs (l1, 2m) and (l1, 2m + 1) of multi-index t for every l1;
//   U is staged as [l1][i][l2] so that one 16-byte LDS read feeds both.
// PAIR_INNER (otherwise): unit u computes multi-indices t = 2u and 2u + 1,
//   which differ in the innermost multi-index dim (output stride 1); every U
//   entry read from LDS feeds two FMAs.
// The host checks that every pair starts at an even offset and stays inside
// one packed 32-k piece (iso_pairs_ok).
template <bool PAIR_RUN, int N>
__global__ void __launch_bounds__(kThreads) iso_expand_pairs_kernel(ExpandParams p, const double *__restrict__ in,
                                                                    const double *__restrict__ U,
                                                                    uint16_t *__restrict__ hi,
                                                                    uint16_t *__restrict__ lo) {
    extern __shared__ __align__(16) double sUp[];
    const int nU = p.L1 * N * N;
    for (int idx = threadIdx.x; idx < nU; idx += blockDim.x) {
        const int c = idx % N, b = (idx / N) % N, l1 = idx / (N * N);
        // PAIR_RUN: [l1][i = b][l2 = c]; PAIR_INNER: [l1][l2 = b][i = c]
        sUp[idx] = PAIR_RUN ? U[l1 * p.u1 + c * p.u2 + b * p.us] : U[l1 * p.u1 + b * p.u2 + c * p.us];
    }
    __syncthreads();
    constexpr uint32_t NP = N / 2;
    const uint32_t units = PAIR_RUN ? p.threads * NP : p.threads / 2;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < units; u += gridDim.x * blockDim.x) {
        const uint32_t t = PAIR_RUN ? u / NP : 2 * u;
        const uint32_t m2 = PAIR_RUN ? 2 * (u - t * NP) : 0;
        uint32_t rem = t, ib = 0, ob = 0;
        for (int k = p.nd - 1; k >= 0; --k) {
            uint32_t q = fast_div(rem, p.ext[k]);
            uint32_t c = rem - q * p.ext[k].d;
            ib += c * p.in_st[k];
            ob += c * p.out_st[k];
            rem = q;
        }
        if (PAIR_RUN) {
            double v[N];
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = in[ib + i * p.xs];
#pragma unroll 1
            for (int l1 = 0; l1 < p.L1; ++l1) {
                const double *ul = sUp + l1 * N * N + m2;
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const double2 w = *(const double2 *)(ul + i * N);
                    a0 = fma(w.x, v[i], a0);
                    a1 = fma(w.y, v[i], a1);
                }
                const uint16_t h0 = bf16_bits((float)a0), w0 = bf16_bits((float)(a0 - bf16_value(h0)));
                const uint16_t h1 = bf16_bits((float)a1), w1 = bf16_bits((float)(a1 - bf16_value(h1)));
                const size_t q0 = split_offset(p, ob + l1 * p.o1 + m2);
                *(uint32_t *)(hi + q0) = (uint32_t)h0 | ((uint32_t)h1 << 16);
                *(uint32_t *)(lo + q0) = (uint32_t)w0 | ((uint32_t)w1 << 16);
            }
        } else {
            const uint32_t ib1 = ib + p.in_st[p.nd - 1];
            double v0[N], v1[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                v0[i] = in[ib + i * p.xs];
                v1[i] = in[ib1 + i * p.xs];
            }
#pragma unroll 1
            for (int l1 = 0; l1 < p.L1; ++l1) {
#pragma unroll 1
                for (int l2 = 0; l2 < N; ++l2) {
                    const double *ul = sUp + (l1 * N + l2) * N;
                    double a0 = 0.0, a1 = 0.0;
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        a0 = fma(ul[i], v0[i], a0);
                        a1 = fma(ul[i], v1[i], a1);
                    }
                    const uint16_t h0 = bf16_bits((float)a0), w0 = bf16_bits((float)(a0 - bf16_value(h0)));
                    const uint16_t h1 = bf16_bits((float)a1), w1 = bf16_bits((float)(a1 - bf16_value(h1)));
                    const size_t q0 = split_offset(p, ob + l1 * p.o1 + l2 * p.o2);
                    *(uint32_t *)(hi + q0) = (uint32_t)h0 | ((uint32_t)h1 << 16);
                    *(uint32_t *)(lo + q0) = (uint32_t)w0 | ((uint32_t)w1 << 16);
                }
            }
        }
    }
}

// Whether the paired kernel applies: every pair's first offset is even (so the
// pair is one aligned 4-byte word of one row, and, in the packed layout, of one
// 32-k piece), and the unit count fits 32 bits.
bool iso_pairs_ok(const ExpandParams &p, bool run) {
    if (p.nsum != p.L2 || p.L2 % 2 != 0 || p.L2 > 12 || p.nd < 1) return false;
    if ((size_t)p.L1 * p.L2 * p.L2 * sizeof(double) > 48 * 1024) return false;
    if (p.pack && p.pld.d % 2 != 0) return false;
    if (p.L1 > 1 && p.o1 % 2 != 0) return false;
    if (run) {
        for (int k = 0; k < p.nd; ++k)
            if (p.out_st[k] % 2 != 0) return false;
        return (uint64_t)p.threads * (p.L2 / 2) < (1ull << 32);
    }
    if (p.o2 % 2 != 0 || p.out_st[p.nd - 1] != 1 || p.ext[p.nd - 1].d % 2 != 0) return false;
    for (int k = 0; k < p.nd - 1; ++k)
        if (p.out_st[k] % 2 != 0) return false;
    return true;
}

template <int N>
void launch_iso_expand_pairs(const ExpandParams &p, bool run, const double *in, const double *U, uint16_t *hi,
                             uint16_t *lo, hipStream_t s) {
    const size_t lds = (size_t)p.L1 * N * N * sizeof(double);
    const uint64_t units = run ? (uint64_t)p.threads * (N / 2) : p.threads / 2;
    const int g = grid_for(units, kThreads, 4096);
    if (run) iso_expand_pairs_kernel<true, N><<<g, kThreads, lds, s>>>(p, in, U, hi, lo);
    else iso_expand_pairs_kernel<false, N><<<g, kThreads, lds, s>>>(p, in, U, hi, lo);
}

void launch_iso_expand(const ExpandParams &pin, const double *in, const double *U, double *out, uint16_t *hi,
                       uint16_t *lo, hipStream_t s) {
    if (pin.threads == 0) return;
    if (pin.z2 == 4) {
        // transposed block scatter; the host checks nsum == L2 <= 13 and the LDS size
        const bool split = pin.zhi[0] != nullptr;
        switch (pin.L2) {
            case 1: return launch_iso_expand_z2t<1>(pin, split, in, U, s);
            case 2: return launch_iso_expand_z2t<2>(pin, split, in, U, s);
            case 3: return launch_iso_expand_z2t<3>(pin, split, in, U, s);
            case 4: return launch_iso_expand_z2t<4>(pin, split, in, U, s);
            case 5: return launch_iso_expand_z2t<5>(pin, split, in, U, s);
            case 6: return launch_iso_expand_z2t<6>(pin, split, in, U, s);
            case 7: return launch_iso_expand_z2t<7>(pin, split, in, U, s);
            case 8: return launch_iso_expand_z2t<8>(pin, split, in, U, s);
            case 9: return launch_iso_expand_z2t<9>(pin, split, in, U, s);
            case 10: return launch_iso_expand_z2t<10>(pin, split, in, U, s);
            case 11: return launch_iso_expand_z2t<11>(pin, split, in, U, s);
            case 12: return launch_iso_expand_z2t<12>(pin, split, in, U, s);
            case 13: return launch_iso_expand_z2t<13>(pin, split, in, U, s);
            default: return;
        }
    }
    if (pin.z2) {
        // the host checks nsum == L2 <= 13 and the LDS size (z2_expand_ok)
        const bool split = pin.zhi[0] != nullptr;
        switch (pin.L2) {
            case 1: return launch_iso_expand_z2<1>(pin, split, in, U, s);
            case 2: return launch_iso_expand_z2<2>(pin, split, in, U, s);
            case 3: return launch_iso_expand_z2<3>(pin, split, in, U, s);
            case 4: return launch_iso_expand_z2<4>(pin, split, in, U, s);
            case 5: return launch_iso_expand_z2<5>(pin, split, in, U, s);
            case 6: return launch_iso_expand_z2<6>(pin, split, in, U, s);
            case 7: return launch_iso_expand_z2<7>(pin, split, in, U, s);
            case 8: return launch_iso_expand_z2<8>(pin, split, in, U, s);
            case 9: return launch_iso_expand_z2<9>(pin, split, in, U, s);
            case 10: return launch_iso_expand_z2<10>(pin, split, in, U, s);
            case 11: return launch_iso_expand_z2<11>(pin, split, in, U, s);
            case 12: return launch_iso_expand_z2<12>(pin, split, in, U, s);
            case 13: return launch_iso_expand_z2<13>(pin, split, in, U, s);
            default: return;
        }
    }
    // The two output loops enter the product symmetrically; when the first
    // one has unit output stride, exchange them so that the run kernels
    // (unit stride on the second loop) apply.
    ExpandParams p = pin;
    if (p.o1 == 1 && p.o2 != 1 && p.L1 > 1 && p.nsum == p.L1) {
        std::swap(p.L1, p.L2);
        std::swap(p.u1, p.u2);
        std::swap(p.o1, p.o2);
    }
    if (hi && ((uintptr_t)hi & 3) == 0 && ((uintptr_t)lo & 3) == 0 && iso_pairs_ok(p, p.o2 == 1)) {
        const bool run = p.o2 == 1;
        switch (p.L2) {
            case 2: return launch_iso_expand_pairs<2>(p, run, in, U, hi, lo, s);
            case 4: return launch_iso_expand_pairs<4>(p, run, in, U, hi, lo, s);
            case 6: return launch_iso_expand_pairs<6>(p, run, in, U, hi, lo, s);
            case 8: return launch_iso_expand_pairs<8>(p, run, in, U, hi, lo, s);
            case 10: return launch_iso_expand_pairs<10>(p, run, in, U, hi, lo, s);
            case 12: return launch_iso_expand_pairs<12>(p, run, in, U, hi, lo, s);
            default: break;
        }
    }
    if (p.nsum == p.L2 && (size_t)p.L1 * p.L2 * p.L2 * sizeof(double) <= 48 * 1024) {
        switch (p.L2) {
            case 2: return launch_iso_expand_lds<2>(p, in, U, out, hi, lo, s);
            case 3: return launch_iso_expand_lds<3>(p, in, U, out, hi, lo, s);
            case 4: return launch_iso_expand_lds<4>(p, in, U, out, hi, lo, s);
            case 5: return launch_iso_expand_lds<5>(p, in, U, out, hi, lo, s);
            case 6: return launch_iso_expand_lds<6>(p, in, U, out, hi, lo, s);
            case 7: return launch_iso_expand_lds<7>(p, in, U, out, hi, lo, s);
            case 8: return launch_iso_expand_lds<8>(p, in, U, out, hi, lo, s);
            case 9: return launch_iso_expand_lds<9>(p, in, U, out, hi, lo, s);
            case 10: return launch_iso_expand_lds<10>(p, in, U, out, hi, lo, s);
            case 11: return launch_iso_expand_lds<11>(p, in, U, out, hi, lo, s);
            case 12: return launch_iso_expand_lds<12>(p, in, U, out, hi, lo, s);
            case 13: return launch_iso_expand_lds<13>(p, in, U, out, hi, lo, s);
            default: break;
        }
    }
    const int g = grid_for(p.threads);
    const bool run = p.o2 == 1 && p.L2 > 1;
    if (hi) {
        if (run) iso_expand_kernel<true, true><<<g, kThreads, 0, s>>>(p, in, U, out, hi, lo);
        else iso_expand_kernel<true, false><<<g, kThreads, 0, s>>>(p, in, U, out, hi, lo);
    } else {
        if (run) iso_expand_kernel<false, true><<<g, kThreads, 0, s>>>(p, in, U, out, hi, lo);
        else iso_expand_kernel<false, false><<<g, kThreads, 0, s>>>(p, in, U, out, hi, lo);
    }
}

// ---------------------------------------------------------------------------
// Z2 block form -> canonical tensor (see Z2UnpackParams).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) z2_unpack_kernel(Z2UnpackParams p, double *__restrict__ out,
                                                             double scale) {
    for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < p.total; o += gridDim.x * blockDim.x) {
        uint32_t rem = o, r = 0, c = 0;
        for (int k = p.nd - 1; k >= 0; --k) {
            const uint32_t q = fast_div(rem, p.ext[k]);
            const uint32_t d = rem - q * p.ext[k].d;
            r += d * p.rst[k];
            c += d * p.cst[k];
            rem = q;
        }
        const uint32_t rt = p.rtab[r], ct = p.rtab[c];
        const uint32_t g = ct >> 31;
        double v = 0.0;
        if (((rt >> 31) ^ g) == p.P)
            v = scale * p.C[g][(size_t)(p.row_off[g] + (rt & ~Z2_PAR)) * p.N[g] + (ct & ~Z2_PAR)];
        out[o] = v;
    }
}

void launch_z2_unpack(const Z2UnpackParams &p, double *out, double scale, hipStream_t s) {
    if (p.total == 0) return;
    z2_unpack_kernel<<<grid_for(p.total), kThreads, 0, s>>>(p, out, scale);
}

// ---------------------------------------------------------------------------
// Deterministic sum of squares.
// ---------------------------------------------------------------------------
__device__ double block_sum(double v, double *sh) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kThreads) sumsq_partial_kernel(const double *__restrict__ x, size_t n,
                                                                 double *__restrict__ partials) {
    __shared__ double sh[kThreads];
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc = fma(x[i], x[i], acc);
    double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ void __launch_bounds__(1024) sum_final_kernel(const double *__restrict__ partials, int n,
                                                         double *__restrict__ out) {
    __shared__ double sh[1024];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partials[i];
    double r = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = r;
}

void launch_sumsq(const double *x, size_t n, double *partials, int npartials, double *out, hipStream_t s) {
    int g = npartials;
    sumsq_partial_kernel<<<g, kThreads, 0, s>>>(x, n, partials);
    sum_final_kernel<<<1, 1024, 0, s>>>(partials, g, out);
}

// ---------------------------------------------------------------------------
// Traces (Eq. (2.5)) and the A matrix of Eq. (3.2).
// ---------------------------------------------------------------------------
struct TraceDims {
    int D[4];
    uint32_t diag_st[4];  // stride of moving both legs of an axis by one
    uint32_t leg_st[8];
};

__global__ void __launch_bounds__(kThreads) trace_obs_kernel(const double *__restrict__ T0,
                                                             const double *__restrict__ T1,
                                                             const double *__restrict__ T2, TraceDims td,
                                                             int axis, double *__restrict__ out) {
    __shared__ double sh[kThreads];
    int b = blockIdx.x;
    if (b < 3) {
        const double *T = b == 0 ? T0 : (b == 1 ? T1 : T2);
        if (!T) {
            if (threadIdx.x == 0) out[b] = 0.0;
            return;
        }
        uint32_t total = (uint32_t)td.D[0] * td.D[1] * td.D[2] * td.D[3];
        double acc = 0.0;
        for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
            uint32_t rem = e, off = 0;
            for (int q = 3; q >= 0; --q) {
                off += (rem % td.D[q]) * td.diag_st[q];
                rem /= td.D[q];
            }
            acc += T[off];
        }
        double r = block_sum(acc, sh);
        if (threadIdx.x == 0) out[b] = r;
        return;
    }
    // A[t, t'] for t, t' of `axis`; sum over the diagonals of the other axes
    int e = b - 3;
    int Da = td.D[axis];
    int t = e / Da, tp = e % Da;
    uint32_t base = t * td.leg_st[2 * axis] + tp * td.leg_st[2 * axis + 1];
    uint32_t total = 1;
    for (int q = 0; q < 4; ++q)
        if (q != axis) total *= td.D[q];
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < total; i += blockDim.x) {
        uint32_t rem = i, off = base;
        for (int q = 3; q >= 0; --q) {
            if (q == axis) continue;
            off += (rem % td.D[q]) * td.diag_st[q];
            rem /= td.D[q];
        }
        acc += T0[off];
    }
    double r = block_sum(acc, sh);
    if (threadIdx.x == 0) out[3 + e] = r;
}

void launch_trace_obs(const double *T0, const double *T1, const double *T2, const int D[4], int axis,
                      double *out, hipStream_t s) {
    TraceDims td;
    uint32_t st = 1;
    for (int l = 7; l >= 0; --l) {
        td.leg_st[l] = st;
        st *= (uint32_t)D[l / 2];
    }
    for (int q = 0; q < 4; ++q) {
        td.D[q] = D[q];
        td.diag_st[q] = td.leg_st[2 * q] + td.leg_st[2 * q + 1];
    }
    int nblocks = 3 + D[axis] * D[axis];
    trace_obs_kernel<<<nblocks, kThreads, 0, s>>>(T0, T1, T2, td, axis, out);
}

// ---------------------------------------------------------------------------
// Gram of the rows of X (R x K, row-major): split-K partial products.  The
// R x R output is covered by tiles of GR_TILE x GR_TILE (blockIdx.y), each
// computed by a 16 x 16 thread grid owning up to 9 x 9 outputs; the two row
// ranges of a tile are staged in LDS per 16-k step.  Every output is one FMA
// chain over its chunk's k in increasing order, whatever the tiling.
// ---------------------------------------------------------------------------
constexpr int GR_MAXB = 9;
constexpr int GR_TILE = 16 * GR_MAXB;  // 144
constexpr int GR_KB = 16;
constexpr int GR_MAXR = 2 * GR_TILE;   // R <= 288 (environments up to 169 rows)

__global__ void __launch_bounds__(256) gram_partial_kernel(const double *__restrict__ X, int R, size_t K,
                                                          size_t chunk, int ntile, double *__restrict__ partials) {
    __shared__ double Xa[GR_TILE][GR_KB + 1];
    __shared__ double Xb[GR_TILE][GR_KB + 1];
    const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
    const int r0 = (blockIdx.y / ntile) * GR_TILE, c0 = (blockIdx.y % ntile) * GR_TILE;
    const int Ra = min(GR_TILE, R - r0), Rb = min(GR_TILE, R - c0);
    size_t k0 = (size_t)blockIdx.x * chunk;
    size_t k1 = k0 + chunk < K ? k0 + chunk : K;
    double acc[GR_MAXB][GR_MAXB];
#pragma unroll
    for (int a = 0; a < GR_MAXB; ++a)
#pragma unroll
        for (int b = 0; b < GR_MAXB; ++b) acc[a][b] = 0.0;
    for (size_t kb = k0; kb < k1; kb += GR_KB) {
        for (int idx = threadIdx.x; idx < GR_TILE * GR_KB; idx += 256) {
            int r = idx / GR_KB, kk = idx % GR_KB;
            size_t k = kb + kk;
            Xa[r][kk] = (k < k1 && r < Ra) ? X[(size_t)(r0 + r) * K + k] : 0.0;
            Xb[r][kk] = (k < k1 && r < Rb) ? X[(size_t)(c0 + r) * K + k] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < GR_KB; ++kk) {
            double xa[GR_MAXB], xb[GR_MAXB];
#pragma unroll
            for (int a = 0; a < GR_MAXB; ++a) {
                xa[a] = Xa[ti + 16 * a][kk];
                xb[a] = Xb[tj + 16 * a][kk];
            }
#pragma unroll
            for (int a = 0; a < GR_MAXB; ++a)
#pragma unroll
                for (int b = 0; b < GR_MAXB; ++b) acc[a][b] = fma(xa[a], xb[b], acc[a][b]);
        }
        __syncthreads();
    }
    double *P = partials + (size_t)blockIdx.x * R * R;
#pragma unroll
    for (int a = 0; a < GR_MAXB; ++a)
#pragma unroll
        for (int b = 0; b < GR_MAXB; ++b) {
            int r = ti + 16 * a, c = tj + 16 * b;
            if (r < Ra && c < Rb) P[(size_t)(r0 + r) * R + c0 + c] = acc[a][b];
        }
}

__global__ void __launch_bounds__(kThreads) gram_reduce_kernel(const double *__restrict__ partials, int RR,
                                                               int nchunks, double *__restrict__ G) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= RR) return;
    double acc = 0.0;
    for (int c = 0; c < nchunks; ++c) acc += partials[(size_t)c * RR + e];
    G[e] = acc;
}

void launch_gram(const double *X, int R, size_t K, double *partials, int nchunks, double *G, hipStream_t s) {
    if (R <= 0 || R > GR_MAXR) return;  // the host checks R (engine: at most 169)
    size_t chunk = (K + nchunks - 1) / nchunks;
    chunk = (chunk + GR_KB - 1) / GR_KB * GR_KB;
    int used = (int)((K + chunk - 1) / chunk);
    const int ntile = (R + GR_TILE - 1) / GR_TILE;
    gram_partial_kernel<<<dim3(used, ntile * ntile), 256, 0, s>>>(X, R, K, chunk, ntile, partials);
    gram_reduce_kernel<<<grid_for((size_t)R * R), kThreads, 0, s>>>(partials, R * R, used, G);
}

// ---------------------------------------------------------------------------
// Squeezed environment E[(p q), (p' q')] = sum_{a a'} G1[p a p' a'] G2[q a q' a'].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) env_combine_kernel(const double *__restrict__ G1,
                                                               const double *__restrict__ G2, int Dp, int Dq,
                                                               int Da, double *__restrict__ E) {
    int n = Dp * Dq;
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    int row = e / n, col = e % n;
    int p = row / Dq, q = row % Dq, pp = col / Dq, qq = col % Dq;
    int R1 = Dp * Da, R2 = Dq * Da;
    double acc = 0.0;
    for (int a = 0; a < Da; ++a)
        for (int ap = 0; ap < Da; ++ap)
            acc = fma(G1[(size_t)(p * Da + a) * R1 + pp * Da + ap], G2[(size_t)(q * Da + a) * R2 + qq * Da + ap],
                      acc);
    E[e] = acc;
}

void launch_env_combine(const double *G1, const double *G2, int Dp, int Dq, int Da, double *E, hipStream_t s) {
    int n = Dp * Dq;
    env_combine_kernel<<<grid_for((size_t)n * n), kThreads, 0, s>>>(G1, G2, Dp, Dq, Da, E);
}

__global__ void identity_kernel(double *U, int n) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n * n) U[e] = (e / n == e % n) ? 1.0 : 0.0;
}

void launch_identity(double *U, int n, hipStream_t s) {
    identity_kernel<<<grid_for((size_t)n * n), kThreads, 0, s>>>(U, n);
}

__global__ void zero_kernel(double *x, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

// FP64 rows [R][K] (row stride K) -> bf16 hi / lo in the packed GEMM layout
// with row length ld >= K; the padding columns K .. ld - 1 are written as 0.
__global__ void __launch_bounds__(kThreads) split_pack_kernel(const double *__restrict__ X, uint32_t R, uint32_t K,
                                                              FastDiv ld, uint32_t pkb, uint16_t *__restrict__ hi,
                                                              uint16_t *__restrict__ lo) {
    const size_t total = (size_t)R * ld.d;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const uint32_t r = (uint32_t)(idx / ld.d), k = (uint32_t)(idx - (size_t)r * ld.d);
        const double v = k < K ? X[(size_t)r * K + k] : 0.0;
        const uint16_t h = bf16_bits((float)v);
        const size_t po = ((size_t)(r / PACK_ROWS) * pkb + k / PACK_K) * (PACK_ROWS * PACK_K) +
                          (r % PACK_ROWS) * PACK_K + k % PACK_K;
        hi[po] = h;
        lo[po] = bf16_bits((float)(v - bf16_value(h)));
    }
}

void launch_split_pack(const double *X, uint32_t R, uint32_t K, uint32_t ld, uint16_t *hi, uint16_t *lo,
                       hipStream_t s) {
    if (R == 0 || ld == 0) return;
    split_pack_kernel<<<grid_for((size_t)R * ld), kThreads, 0, s>>>(X, R, K, make_fastdiv(ld), ld / PACK_K, hi, lo);
}

void launch_zero(double *x, size_t n, hipStream_t s) {
    if (n == 0) return;
    zero_kernel<<<grid_for(n), kThreads, 0, s>>>(x, n);
}

}  // namespace hotrg
