// Deterministic FP64 reductions used by the Davidson solver.
//
// Inner products G = X Y^T of a few long vectors are a GEMM with a huge K: the K
// axis is cut into fixed chunks, each chunk is one batch of the matrix-core GEMM
// (so every vector element is read once), and the per-chunk partial Gram blocks
// are summed in a fixed order -- the result does not depend on scheduling.
#include "internal.h"

namespace adc3 {

namespace {
constexpr long long CHUNK = 4096;

__global__ void sum_partials_kernel(const double* partial, long long nchunk, int np, int nq, double* G, int ldg) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np * nq) return;
    int p = t / nq, q = t % nq;
    double acc = 0.0;
    for (long long c = 0; c < nchunk; ++c) acc += partial[c * np * nq + t];
    G[p * ldg + q] = acc;
}
}  // namespace

size_t dots_partial_elems(int np, int nq, long long n) { return (size_t)(n / CHUNK + 2) * np * nq; }

void k_dots(const double* X, long long ldx, int np, const double* Y, long long ldy, int nq, long long n, double* G,
            int ldg, double* partial, hipStream_t s) {
    if (g_dry) return;
    if (np <= 0 || nq <= 0) return;
    long long nfull = n / CHUNK, rem = n % CHUNK;
    long long nchunk = nfull + (rem ? 1 : 0);
    if (nchunk == 0) {
        // empty vectors: G = 0
        k_fill(partial, (long long)np * nq, 0.0, s);
        nchunk = 1;
    }
    const long long pq = (long long)np * nq;
    // partial buffer holds nchunk * np * nq doubles (caller sizes it with dots_partial_elems)
    for (long long c0 = 0; c0 < nfull; c0 += 65535) {
        long long nb = std::min<long long>(65535, nfull - c0);
        Gemm g;
        g.M = np; g.N = nq; g.K = (int)CHUNK;
        g.A = X + c0 * CHUNK; g.sAm = ldx; g.sAk = 1; g.bA0 = CHUNK;
        g.B = Y + c0 * CHUNK; g.sBk = 1; g.sBn = ldy; g.bB0 = CHUNK;
        g.C = partial + c0 * pq; g.sCm = nq; g.sCn = 1; g.bC0 = pq;
        g.nb0 = (int)nb;
        gemm(g, s);
    }
    if (rem) {
        Gemm g;
        g.M = np; g.N = nq; g.K = (int)rem;
        g.A = X + nfull * CHUNK; g.sAm = ldx; g.sAk = 1;
        g.B = Y + nfull * CHUNK; g.sBk = 1; g.sBn = ldy;
        g.C = partial + nfull * pq; g.sCm = nq; g.sCn = 1;
        gemm(g, s);
    }
    hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)((pq + 255) / 256)), dim3(256), 0, s, partial, nchunk,
                       np, nq, G, ldg);
    LAUNCHCHK();
}

void k_lincomb(double* Y, long long ldy, int nq, const double* X, long long ldx, int np, const double* C, int ldc,
               long long n, double alpha, double beta, hipStream_t s) {
    if (g_dry) return;
    if (nq <= 0 || n <= 0) return;
    for (long long c0 = 0; c0 < n; c0 += 2000000000LL) {
        long long nn = std::min<long long>(n - c0, 2000000000LL);
        Gemm g;
        g.M = nq; g.N = (int)nn; g.K = np;
        g.A = C; g.sAm = 1; g.sAk = ldc;
        g.B = X + c0; g.sBk = ldx; g.sBn = 1;
        g.C = Y + c0; g.sCm = ldy; g.sCn = 1;
        g.alpha = alpha; g.beta = beta;
        gemm(g, s);
    }
}

}  // namespace adc3
