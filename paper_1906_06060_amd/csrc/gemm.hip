// Contraction GEMMs of the HOTRG step.
//
//   C[M x N] (+)= A[M x K] * B[N x K]^T,   both operands K-contiguous.
//
// The O(D^15) contraction of Sec. 2 (cost paragraph) is exactly this
// product with M = N = D^4 and K = D^7 (taken in K slices):
//   * gemm_f64:    FP64 on the vector FMA units (under load they sustain
//                  about 1.3x the rate of v_mfma_f64_16x16x4 measured in
//                  register-only loops), 128 x 128 tile, 8 x 8 outputs per
//                  thread, operands staged k-major in a two-slot LDS ring;
//   * gemm_bf16x3: v_mfma_f32_32x32x16_bf16 on hi/lo splits (3 products),
//                  256 x 256 tile, 8 waves of 128 x 64 (two per SIMD), 32 k
//                  per LDS stage loaded directly into a two-slot LDS ring
//                  (operands in a packed, stage-contiguous layout), FP32
//                  accumulation inside chunks of 32768 k; each chunk is added
//                  into the FP64 output tile (owned by one workgroup, so no
//                  atomics).
// Tiles are ordered so that the blocks an XCD runs together form a compact
// patch of the output (shared A rows / B columns stay in that XCD's L2).
#include "hotrg_internal.h"

#include <algorithm>

namespace hotrg {

typedef float flt16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Round-robin XCD dispatch undone: consecutive units run on one XCD.
__device__ __forceinline__ int unit_of(int bid, int nb) {
    const int full = nb - nb % 8;
    return bid < full ? (bid % 8) * (full / 8) + bid / 8 : bid;
}

// Tile index t -> (tile row, tile col): groups of `G` tile rows walked column
// by column.
__device__ __forceinline__ void tile_rc(int t, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int G = 8;
    const int per_group = G * tiles_n;
    const int group = t / per_group;
    const int first = group * G;
    const int gsize = min(tiles_m - first, G);
    const int r = t % per_group;
    tm = first + r % gsize;
    tn = r / gsize;
}

// blockIdx.x -> (tile row, tile col) for a launch covering every tile.
__device__ __forceinline__ void tile_of(int bid, int tiles_m, int tiles_n, int &tm, int &tn) {
    tile_rc(unit_of(bid, tiles_m * tiles_n), tiles_m, tiles_n, tm, tn);
}

// ------------------------------------------------------------------ FP64 ---
namespace f64 {
constexpr int BM = 128, BN = 128, BK = 8, PAD = 4, NT = 256;
constexpr int PER = BK / 2;  // k values each thread stages per operand and stage

// Register-blocked DGEMM: a 16 x 16 thread grid, each thread owns the row
// pairs 2 ty + 32 i + {0, 1} and the column pairs 2 tx + 32 j + {0, 1}
// (i, j < 4); operands staged k-major in a two-slot LDS ring, so every
// operand pair is one 16-byte LDS read (a wave reads 4 broadcast A pairs and
// 16 consecutive B pairs per k) and there is one barrier per stage: stage
// s + 1 is fetched into registers while stage s is multiplied, then written
// to the other slot.  Thread t stages k values [PER (t & 1), PER (t & 1) +
// PER) of tile row t / 2; with VEC (both leading dimensions even, operands
// 16-byte aligned) those are 16-byte loads, which measured 11-13% faster
// than 8-byte ones on the contraction shapes.  The sum over k runs in
// ascending order in every variant.
template <bool VEC>
__global__ void __launch_bounds__(NT) gemm_f64_kernel(const double *__restrict__ A, const double *__restrict__ B,
                                                       double *__restrict__ C, int M, int N, int K, size_t lda,
                                                       size_t ldb, size_t ldc, int accumulate, int tiles_m,
                                                       int tiles_n) {
    __shared__ __align__(16) double As[2][BK][BM + PAD];
    __shared__ __align__(16) double Bs[2][BK][BN + PAD];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    int tm, tn;
    tile_of(blockIdx.x, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int lr = tid >> 1, kp = (tid & 1) * PER;
    const bool arow = (m0 + lr) < M, brow = (n0 + lr) < N;
    const double *Ap = A + (size_t)(arow ? m0 + lr : 0) * lda;
    const double *Bp = B + (size_t)(brow ? n0 + lr : 0) * ldb;
    double acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
    double ra[PER], rb[PER];
    auto gload = [&](int k0) {
        const int kb = k0 + kp;
        if (VEC && kb + PER <= K) {
#pragma unroll
            for (int j = 0; j < PER; j += 2) {
                const double2 va = arow ? *(const double2 *)(Ap + kb + j) : double2{0.0, 0.0};
                const double2 vb = brow ? *(const double2 *)(Bp + kb + j) : double2{0.0, 0.0};
                ra[j] = va.x;
                ra[j + 1] = va.y;
                rb[j] = vb.x;
                rb[j + 1] = vb.y;
            }
        } else {
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int k = kb + j;
                ra[j] = (arow && k < K) ? Ap[k] : 0.0;
                rb[j] = (brow && k < K) ? Bp[k] : 0.0;
            }
        }
    };
    auto lstore = [&](int slot) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            As[slot][kp + j][lr] = ra[j];
            Bs[slot][kp + j][lr] = rb[j];
        }
    };
    const int ns = (K + BK - 1) / BK;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
        const int cur = s & 1;
        if (s + 1 < ns) gload((s + 1) * BK);
#pragma unroll 2
        for (int kk = 0; kk < BK; ++kk) {
            double a[8], b[8];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double2 va = *(const double2 *)&As[cur][kk][2 * ty + 32 * i];
                const double2 vb = *(const double2 *)&Bs[cur][kk][2 * tx + 32 * i];
                a[2 * i] = va.x;
                a[2 * i + 1] = va.y;
                b[2 * i] = vb.x;
                b[2 * i + 1] = vb.y;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        // the other slot was last read in stage s - 1, before the barrier
        // that ended it; the barrier below publishes it for stage s + 1
        if (s + 1 < ns) lstore(cur ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int row = m0 + 2 * ty + 32 * (i >> 1) + (i & 1);
        if (row >= M) continue;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int col = n0 + 2 * tx + 32 * (j >> 1) + (j & 1);
            if (col < N) {
                double *c = C + (size_t)row * ldc + col;
                *c = accumulate ? *c + acc[i][j] : acc[i][j];
            }
        }
    }
}
}  // namespace f64

void launch_gemm_f64(const double *A, const double *B, double *C, int M, int N, int K, size_t lda, size_t ldb,
                     size_t ldc, int accumulate, hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    int tm = (M + f64::BM - 1) / f64::BM, tn = (N + f64::BN - 1) / f64::BN;
    const bool vec = lda % 2 == 0 && ldb % 2 == 0 && (uintptr_t)A % 16 == 0 && (uintptr_t)B % 16 == 0;
    if (vec)
        f64::gemm_f64_kernel<true><<<tm * tn, f64::NT, 0, s>>>(A, B, C, M, N, K, lda, ldb, ldc, accumulate, tm, tn);
    else
        f64::gemm_f64_kernel<false><<<tm * tn, f64::NT, 0, s>>>(A, B, C, M, N, K, lda, ldb, ldc, accumulate, tm,
                                                                tn);
}

// ---------------------------------------------------------------- bf16x3 ---
namespace x3 {
constexpr int BM = 256, BN = 256;
constexpr int BK = PACK_K;   // k per LDS stage: one packed block of every operand
constexpr int NT = 512;      // eight waves, two per SIMD, each 128 x 64 of the tile
constexpr int KC = 32768;    // k per FP32 accumulation chunk (each flush read-modify-writes the FP64 tile)
constexpr size_t OPB = (size_t)BM * BK * sizeof(uint16_t);  // one operand block: 16 KB
constexpr size_t STAGE = 4 * OPB;                            // Ah, Al, Bh, Bl: 64 KB
constexpr size_t LDS_FLUSH = (size_t)8 * 32 * 65 * sizeof(float);
constexpr size_t LDS_BYTES = std::max(2 * STAGE, LDS_FLUSH);  // two-slot ring
static_assert(KC % BK == 0, "a chunk is whole stages");

// Operands are packed (see hotrg_internal.h): block (row tile, k block) is a
// contiguous 256 x 32 run (64-byte rows), so one stage of one operand is 16 KB
// of consecutive memory.  It goes straight from global memory into LDS
// (global_load_lds_dwordx4: lane i of a wave writes bytes 16 i .. 16 i + 15 of
// the wave's 1 KB destination), into a two-slot ring: stage s + 1 is in flight
// while stage s is multiplied, with no VGPRs spent on staging.  Lane i of a
// 1 KB chunk (16 rows) fetches piece (i % 4) ^ swz(row) of row i / 4, so LDS
// position (r, p) holds k piece p ^ swz(r), swz(r) = (r / 4) mod 4: the 16
// rows that one group of 16 lanes of a fragment read touches fall into 16
// distinct 16-byte bank groups.
//
// A holds `ntA` tensors of M rows, each padded to Mp = roundup(M, 256); a row
// tile never straddles two tensors and its rows map to C rows t M + r (r < M).
//
// One launch covers the tiles t0 .. t0 + units - 1 of the tile order of up
// to two independent products (tiles below tiles0 belong to the first; a
// launch over both fills the chip with the tiles of both).  With halves = 2
// every tile is two units: k in [0, kmid) added into C as usual, and k in
// [kmid, K) written to the 256 x 256 block `part` + (unit / 2) 2^16, which
// gemm_tail_fixup_kernel adds into C afterwards (used for the last, partly
// filled round of tiles, so that it takes half as long).
struct Prob {
    const uint16_t *Ah, *Al, *Bh, *Bl;
    double *C;
    int M, Mp, N, K;
    size_t ldc;
    int accumulate, tiles_m, tiles_n;
};
struct Launch {
    Prob p[2];
    int tiles0, t0, halves;
    double *part;
};

__global__ void __launch_bounds__(NT) gemm_bf16x3_kernel(const Launch L) {
    extern __shared__ __align__(16) uint16_t smem[];
    char *lds = (char *)smem;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 2, wc = wave & 3;  // wave tile: rows wr*128.., cols wc*64..
    const int u = unit_of(blockIdx.x, gridDim.x);
    const int halves = L.halves;
    const int hf = halves == 2 ? (u & 1) : 0;
    const int tg = L.t0 + (halves == 2 ? (u >> 1) : u);
    const int pi = tg >= L.tiles0 ? 1 : 0;
    const Prob &P = L.p[pi];
    const uint16_t *__restrict__ Ah = P.Ah;
    const uint16_t *__restrict__ Al = P.Al;
    const uint16_t *__restrict__ Bh = P.Bh;
    const uint16_t *__restrict__ Bl = P.Bl;
    double *__restrict__ C = P.C;
    double *__restrict__ part = L.part;
    const int M = P.M, Mp = P.Mp, N = P.N, K = P.K, accumulate = P.accumulate;
    const size_t ldc = P.ldc;
    const int kmid = K / 2 / BK * BK;
    int tm, tn;
    tile_rc(tg - (pi ? L.tiles0 : 0), P.tiles_m, P.tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tens = m0 / Mp, lrow0 = m0 - tens * Mp;  // tensor of this row tile, its first local row
    const int kbeg = hf ? kmid : 0, kend = (halves == 2 && !hf) ? kmid : K;
    // destination of this unit: its C tile (clipped to M x N) or its partial block
    double *const Cd = hf ? part + (size_t)(u >> 1) * (BM * BN) : C + (size_t)(tens * M + lrow0) * ldc + n0;
    const size_t ldd = hf ? (size_t)BN : ldc;
    const int rlim = hf ? BM : M - lrow0, clim = hf ? BN : N - n0;

    // loads: wave w brings half w % 2 (128 rows, 8 KB) of operand w / 2
    const size_t kb = (size_t)K / BK;  // packed k blocks per row tile
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int op = wv >> 1, half = wv & 1;
    const uint16_t *obase = op == 0 ? Ah : (op == 1 ? Al : (op == 2 ? Bh : Bl));
    const char *src0 = (const char *)(obase + (size_t)(op < 2 ? tm : tn) * kb * (BM * BK)) + half * (OPB / 2);
    const uint32_t lsrc = (uint32_t)((lane >> 2) * (BK * 2) + (((lane & 3) ^ ((lane >> 4) & 3)) * 16));
    const uint32_t ldst = (uint32_t)(op * OPB + half * (OPB / 2));
    auto issue = [&](size_t blk, int slot) {
        const char *src = src0 + blk * OPB;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void *)(src + j * 1024 + lsrc),
                (__attribute__((address_space(3))) void *)(lds + slot * STAGE + ldst + j * 1024), 16, 0, 0);
    };

    // fragments: lane l feeds row (or column) l % 32, k 8 (l / 32) .. + 7 of a
    // 16-k substep; the swizzle of rows r + 32 i equals that of r, and substep
    // 1 (pieces 2, 3) is position ^ 2, i.e. byte offset ^ 32
    const int i32 = lane & 31, lq = (lane >> 5) * 4;
    const uint32_t sw = (uint32_t)(((lane >> 5) ^ ((i32 >> 2) & 3)) * 16);
    const uint32_t offA = (uint32_t)(wr * 128 + i32) * (BK * 2) + sw;
    const uint32_t offB = (uint32_t)(2 * OPB) + (uint32_t)(wc * 64 + i32) * (BK * 2) + sw;
    struct Frags {
        bf16x8 ah[4], al[4], bh[2], bl[2];
    };
    auto read = [&](Frags &f, int slot, int sub) {
        const char *b = lds + slot * STAGE;
        const uint32_t x = sub ? 32u : 0u;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            f.bh[j] = *(const bf16x8 *)(b + ((offB ^ x) + j * 32 * (BK * 2)));
            f.bl[j] = *(const bf16x8 *)(b + ((offB ^ x) + j * 32 * (BK * 2) + OPB));
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f.ah[i] = *(const bf16x8 *)(b + ((offA ^ x) + i * 32 * (BK * 2)));
            f.al[i] = *(const bf16x8 *)(b + ((offA ^ x) + i * 32 * (BK * 2) + OPB));
        }
    };

    flt16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
    // D layout of the 32x32 block: lane l, value e -> row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32
    auto mma = [&](const Frags &f) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.al[i], f.bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.ah[i], f.bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.ah[i], f.bh[j], acc[i][j], 0, 0, 0);
            }
    };

    // Add the FP32 partial tile into the FP64 output: in four passes (one per
    // 32-row block of every wave) the accumulators go through LDS and all
    // threads then update C with coalesced row segments.
    bool first = hf ? true : !accumulate;
    float *sC = (float *)smem;
    constexpr int SROW = 65;
    auto flush = [&]() {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float *sw_ = sC + wave * 32 * SROW;
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    sw_[((e >> 2) * 8 + lq + (e & 3)) * SROW + j * 32 + i32] = acc[i][j][e];
                    acc[i][j][e] = 0.0f;
                }
            __syncthreads();
#pragma unroll 2
            for (int q = 0; q < 32; ++q) {
                const int idx = tid + NT * q;
                const int w = idx >> 11, rem = idx & 2047;
                const int rl = rem >> 6, cl = rem & 63;
                const int lr = (w >> 2) * 128 + i * 32 + rl;
                const int lc = (w & 3) * 64 + cl;
                if (lr < rlim && lc < clim) {
                    double *c = Cd + (size_t)lr * ldd + lc;
                    double v = (double)sC[w * 32 * SROW + rl * SROW + cl];
                    *c = first ? v : *c + v;
                }
            }
            __syncthreads();
        }
        first = false;
    };

    // Per stage: the second substep's fragments are read while the first is on
    // the matrix core; one barrier per stage, between the substeps, after which
    // the next stage has landed for every wave and the slot just read may be
    // refilled; the first fragments of the next stage are then read while the
    // second substep runs.  The loop body has no branches (past the end of a
    // chunk the refill reloads a valid block and the fragments read are not
    // used), so the scheduling groups below can place one LDS read (and, in
    // the second substep, one global load) between every two MFMAs.
    for (int kc0 = kbeg; kc0 < kend; kc0 += KC) {
        const int nst = (min(kend, kc0 + KC) - kc0) / BK;
        const size_t b0 = (size_t)kc0 / BK, blast = kb - 1;
        issue(b0, 0);
        __syncthreads();  // (waits for this wave's loads) stage 0 landed everywhere
        issue(min(b0 + 1, blast), 1);
        Frags f0, f1;
        read(f0, 0, 0);
        for (int st = 0; st < nst; ++st) {
            const int slot = st & 1;
            read(f1, slot, 1);
            mma(f0);
#pragma unroll
            for (int g = 0; g < 12; ++g) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // two MFMAs
            }
            __builtin_amdgcn_s_waitcnt(0);  // own loads of stage st + 1, own reads of this slot
            __syncthreads();
            issue(min(b0 + st + 2, blast), slot);
            read(f0, slot ^ 1, 0);
            mma(f1);
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // one global load
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            }
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);  // the last (redundant) refill has landed
        __syncthreads();                // ring reads done before the flush reuses the LDS
        flush();                        // FP32 chunk of at most KC k into the FP64 tile
    }
    if (first) flush();
}

// C tile of split tile s (tile t0 + s of the launch's tile order) += its
// second-half partial block.
__global__ void __launch_bounds__(256) gemm_tail_fixup_kernel(const Launch L) {
    const int s = blockIdx.x;
    const int tg = L.t0 + s;
    const int pi = tg >= L.tiles0 ? 1 : 0;
    const Prob &P = L.p[pi];
    int tm, tn;
    tile_rc(tg - (pi ? L.tiles0 : 0), P.tiles_m, P.tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tens = m0 / P.Mp, lrow0 = m0 - tens * P.Mp;
    const double *p = L.part + (size_t)s * (BM * BN);
    for (int e = threadIdx.x; e < BM * BN; e += blockDim.x) {
        const int lr = e / BN, lc = e % BN;
        if (lrow0 + lr < P.M && n0 + lc < P.N) P.C[(size_t)(tens * P.M + lrow0 + lr) * P.ldc + n0 + lc] += p[e];
    }
}
}  // namespace x3

namespace {
x3::Prob make_prob(const X3Gemm &g) {
    x3::Prob p{};
    p.Ah = g.Ah;
    p.Al = g.Al;
    p.Bh = g.Bh;
    p.Bl = g.Bl;
    p.C = g.C;
    p.M = g.M;
    p.Mp = (g.M + x3::BM - 1) / x3::BM * x3::BM;
    p.N = g.N;
    p.K = g.K;
    p.ldc = g.ldc;
    p.accumulate = g.accumulate;
    p.tiles_m = g.ntA * (p.Mp / x3::BM);
    p.tiles_n = (g.N + x3::BN - 1) / x3::BN;
    return p;
}
}  // namespace

void launch_gemm_bf16x3_multi(const X3Gemm *g, int count, hipStream_t s, double *part) {
    static bool attr_set = false;
    static int ncu = 0;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)x3::gemm_bf16x3_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)x3::LDS_BYTES);
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 0;
        attr_set = true;
    }
    x3::Launch L{};
    int n = 0;
    for (int i = 0; i < count && n < 2; ++i)
        if (g[i].M > 0 && g[i].N > 0 && g[i].ntA > 0 && g[i].K > 0) L.p[n++] = make_prob(g[i]);
    if (n == 0) return;
    if (n == 1) L.p[1] = L.p[0];
    L.tiles0 = L.p[0].tiles_m * L.p[0].tiles_n;
    const int tiles = L.tiles0 + (n == 2 ? L.p[1].tiles_m * L.p[1].tiles_n : 0);
    if (n == 1) L.tiles0 = tiles;
    // One workgroup per CU at a time: the last round of tiles is partly
    // filled.  When it holds at most half the CUs (and there is a full round
    // before it), its tiles run as two k-halves each, after the full rounds
    // (every K is a multiple of 64, so both halves are non-empty).
    const int rem = ncu > 0 ? tiles % ncu : 0;
    if (part && rem > 0 && rem <= ncu / 2 && rem <= GEMM_TAIL_MAX_TILES && tiles > ncu) {
        const int main = tiles - rem;
        L.part = nullptr;
        L.t0 = 0;
        L.halves = 1;
        x3::gemm_bf16x3_kernel<<<main, x3::NT, x3::LDS_BYTES, s>>>(L);
        L.part = part;
        L.t0 = main;
        L.halves = 2;
        x3::gemm_bf16x3_kernel<<<2 * rem, x3::NT, x3::LDS_BYTES, s>>>(L);
        x3::gemm_tail_fixup_kernel<<<rem, 256, 0, s>>>(L);
        return;
    }
    L.part = nullptr;
    L.t0 = 0;
    L.halves = 1;
    x3::gemm_bf16x3_kernel<<<tiles, x3::NT, x3::LDS_BYTES, s>>>(L);
}

void launch_gemm_bf16x3(const uint16_t *Ah, const uint16_t *Al, const uint16_t *Bh, const uint16_t *Bl, double *C,
                        int M, int ntA, int N, int K, size_t ldc, int accumulate, hipStream_t s, double *part) {
    const X3Gemm g{Ah, Al, Bh, Bl, C, M, ntA, N, K, ldc, accumulate};
    launch_gemm_bf16x3_multi(&g, 1, s, part);
}

}  // namespace hotrg
