// FP64 symmetric eigensolver for the environment matrices (n <= 169):
// two-sided cyclic Jacobi with the round-robin ("circle") ordering, so every
// round rotates n/2 disjoint (p, q) planes at once (Golub & Van Loan,
// Matrix Computations, Sec. 8.5: the 2x2 symmetric Schur step and parallel
// orderings).  One workgroup per matrix; the working copies live in global
// memory (they fit in L2).
//
// A plane whose off-diagonal entry is exactly zero is never rotated, so a
// matrix that is block diagonal (for instance in Z2 parity sectors) keeps its
// exact zeros and every eigenvector stays inside one block.
#include "hotrg_internal.h"

namespace hotrg {

constexpr int JT = 512;          // threads per matrix
constexpr int J_MAXN = 170;  // n <= 169, padded to even

__device__ __forceinline__ int rr_player(int pos, int round, int m) {
    // position 0 is fixed, positions 1..m-1 rotate by `round`
    return pos == 0 ? 0 : 1 + (pos - 1 + round) % (m - 1);
}

__device__ double jt_block_sum(double v, double *sh) {
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

__global__ void __launch_bounds__(JT) jacobi_kernel(const double *__restrict__ Ain, int n, double *__restrict__ lam,
                                                    double *__restrict__ Vout, double *__restrict__ work,
                                                    int *__restrict__ sweeps_out, double *__restrict__ resid_out,
                                                    int max_sweeps) {
    __shared__ double cs[J_MAXN / 2 + 1], sn[J_MAXN / 2 + 1];
    __shared__ int pp[J_MAXN / 2 + 1], qq[J_MAXN / 2 + 1];
    __shared__ double red[JT];
    __shared__ double dval[J_MAXN + 1];
    __shared__ int rank[J_MAXN + 1];
    const int mat = blockIdx.x;
    const int m = n + (n & 1);
    const int half = m / 2;
    double *A = work + (size_t)mat * 2 * m * m;
    double *V = A + (size_t)m * m;
    const double *Ai = Ain + (size_t)mat * n * n;
    const int tid = threadIdx.x;

    for (int e = tid; e < m * m; e += JT) {
        int i = e / m, j = e % m;
        A[e] = (i < n && j < n) ? Ai[i * n + j] : 0.0;
        V[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    double fro = 0.0;
    {
        double acc = 0.0;
        for (int e = tid; e < m * m; e += JT) acc += A[e] * A[e];
        fro = jt_block_sum(acc, red);
    }
    int sweep = 0;
    if (m >= 2 && fro > 0.0) {
        for (sweep = 0; sweep < max_sweeps; ++sweep) {
            double off = 0.0;
            {
                double acc = 0.0;
                for (int e = tid; e < m * m; e += JT) {
                    int i = e / m, j = e % m;
                    if (i != j) acc += A[e] * A[e];
                }
                off = jt_block_sum(acc, red);
            }
            if (off <= 1e-30 * fro) break;
            for (int round = 0; round < m - 1; ++round) {
                if (tid < half) {
                    int p = rr_player(tid, round, m), q = rr_player(m - 1 - tid, round, m);
                    if (p > q) {
                        int t = p;
                        p = q;
                        q = t;
                    }
                    double apq = A[p * m + q];
                    double c = 1.0, s = 0.0;
                    if (apq != 0.0) {
                        double app = A[p * m + p], aqq = A[q * m + q];
                        double tau = (aqq - app) / (2.0 * apq);
                        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                    pp[tid] = p;
                    qq[tid] = q;
                    cs[tid] = c;
                    sn[tid] = s;
                }
                __syncthreads();
                // rows: A <- J^T A
                for (int e = tid; e < half * m; e += JT) {
                    int k = e / m, j = e % m;
                    double s = sn[k];
                    if (s == 0.0) continue;
                    double c = cs[k];
                    int p = pp[k], q = qq[k];
                    double ap = A[p * m + j], aq = A[q * m + j];
                    A[p * m + j] = c * ap - s * aq;
                    A[q * m + j] = s * ap + c * aq;
                }
                __syncthreads();
                // columns: A <- A J, V <- V J
                for (int e = tid; e < half * m; e += JT) {
                    int k = e / m, i = e % m;
                    double s = sn[k];
                    if (s == 0.0) continue;
                    double c = cs[k];
                    int p = pp[k], q = qq[k];
                    double ap = A[i * m + p], aq = A[i * m + q];
                    A[i * m + p] = c * ap - s * aq;
                    A[i * m + q] = s * ap + c * aq;
                    double vp = V[i * m + p], vq = V[i * m + q];
                    V[i * m + p] = c * vp - s * vq;
                    V[i * m + q] = s * vp + c * vq;
                }
                __syncthreads();
            }
        }
    }
    // squared off-diagonal norm left, relative to the total (the convergence
    // measure the sweeps test; reported so the host can tell a solve that
    // stopped at the sweep cap from a converged one)
    {
        double acc = 0.0;
        for (int e = tid; e < m * m; e += JT) {
            int i = e / m, j = e % m;
            if (i != j) acc += A[e] * A[e];
        }
        const double off = jt_block_sum(acc, red);
        if (tid == 0 && resid_out) resid_out[mat] = fro > 0.0 ? off / fro : 0.0;
    }
    // sort eigenvalues descending (stable on ties) and emit columns
    for (int i = tid; i < n; i += JT) dval[i] = A[i * m + i];
    __syncthreads();
    for (int i = tid; i < n; i += JT) {
        double di = dval[i];
        int r = 0;
        for (int j = 0; j < n; ++j) {
            double dj = dval[j];
            r += (dj > di) || (dj == di && j < i);
        }
        rank[i] = r;
    }
    __syncthreads();
    for (int i = tid; i < n; i += JT) lam[(size_t)mat * n + rank[i]] = dval[i];
    for (int e = tid; e < n * n; e += JT) {
        int r = e / n, i = e % n;
        Vout[(size_t)mat * n * n + (size_t)r * n + rank[i]] = V[r * m + i];
    }
    if (tid == 0 && sweeps_out) sweeps_out[mat] = sweep;
}

void launch_jacobi_eigh(const double *A, int n, int count, double *lam, double *V, double *work, int *sweeps,
                        double *resid, int max_sweeps, hipStream_t s) {
    if (count <= 0 || n <= 0) return;
    jacobi_kernel<<<count, JT, 0, s>>>(A, n, lam, V, work, sweeps, resid, max_sweeps);
}

}  // namespace hotrg
