// Deterministic FP64 reductions used by the Davidson solver.
//
// Inner products G = X Y^T of a few long vectors are a GEMM with a huge K: the K
// axis is cut into fixed chunks, each chunk is one batch of the matrix-core GEMM
// (every vector element is read once; ~n/1024 workgroups keep the chip busy), and
// the per-chunk partial Gram blocks are summed by one workgroup per output element
// in a fixed order -- the result does not depend on scheduling.
#include "internal.h"
#include <algorithm>

namespace adc3 {

namespace {
inline long long chunk_of(long long n) { return std::max<long long>(256, (n + 8191) / 8192); }

// G[p*ldg + q] = sum_c partial[c][r][s] with (r,s) = (p,q) or (q,p) when swapped
__global__ void sum_partials_kernel(const double* partial, long long nchunk, int M, int N, int swapped, double* G,
                                    int ldg) {
    const int t = blockIdx.x;  // output element of the partial [M][N] block
    const long long MN = (long long)M * N;
    double acc = 0.0;
    for (long long c = threadIdx.x; c < nchunk; c += blockDim.x) acc += partial[c * MN + t];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = red[0] + red[1] + red[2] + red[3];
        int r = t / N, q = t % N;
        if (swapped) G[(long long)q * ldg + r] = s;
        else G[(long long)r * ldg + q] = s;
    }
}
// Small Gram blocks (at most 64 products, e.g. residual norms and the Gram of a new block): one pass
// on the vector ALUs.  Workgroup (c, g) takes elements [c*chunk, (c+1)*chunk) and rows [g*PG, g*PG+PG)
// of X against all nq (<= NQ) rows of Y; the products accumulate in registers, then a fixed-order
// block reduction writes partial[c][p][q].
template <int NQ, int PG>
__global__ __launch_bounds__(256) void dots_small_kernel(const double* X, long long ldx, int np, const double* Y,
                                                         long long ldy, int nq, long long n, long long chunk,
                                                         double* partial) {
    const long long c0 = (long long)blockIdx.x * chunk, c1 = min(n, c0 + chunk);
    const int p0 = blockIdx.y * PG;
    double acc[PG][NQ];
#pragma unroll
    for (int p = 0; p < PG; ++p)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[p][q] = 0.0;
    for (long long t = c0 + threadIdx.x; t < c1; t += 256) {
        double y[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) y[q] = q < nq ? Y[q * ldy + t] : 0.0;
#pragma unroll
        for (int p = 0; p < PG; ++p) {
            if (p0 + p < np) {
                const double x = X[(p0 + p) * ldx + t];
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc[p][q] += x * y[q];
            }
        }
    }
    __shared__ double red[4][PG * NQ];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < PG; ++p)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double v = acc[p][q];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
            if (lane == 0) red[wave][p * NQ + q] = v;
        }
    __syncthreads();
    for (int k = threadIdx.x; k < PG * NQ; k += 256) {
        const int p = k / NQ, q = k % NQ;
        if (p0 + p < np && q < nq)
            partial[((long long)blockIdx.x * np + p0 + p) * nq + q] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// Y[q][t] = alpha * sum_p C[p][q] X[p][t] + beta * Y[q][t] for nq <= NQ rows: each thread E elements
// (stride 256), the coefficients uniform across the wave, X streamed once.
template <int NQ, int E>
__global__ __launch_bounds__(256) void lincomb_kernel(double* Y, long long ldy, int nq, const double* X, long long ldx,
                                                      int np, const double* C, int ldc, long long n, double alpha,
                                                      double beta) {
    const long long base = (long long)blockIdx.x * (256 * E) + threadIdx.x;
    double acc[E][NQ];
#pragma unroll
    for (int e = 0; e < E; ++e)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[e][q] = 0.0;
    for (int p = 0; p < np; ++p) {
        double x[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const long long t = base + 256LL * e;
            x[e] = t < n ? X[p * ldx + t] : 0.0;
        }
        const double* cp = C + (long long)p * ldc;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double c = q < nq ? cp[q] : 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e][q] += c * x[e];
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (q >= nq) break;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const long long t = base + 256LL * e;
            if (t < n) {
                double* y = Y + q * ldy + t;
                *y = alpha * acc[e][q] + (beta == 0.0 ? 0.0 : beta * *y);
            }
        }
    }
}

template <int NQ>
void launch_lincomb(double* Y, long long ldy, int nq, const double* X, long long ldx, int np, const double* C, int ldc,
                    long long n, double alpha, double beta, hipStream_t s) {
    constexpr int E = NQ <= 8 ? 4 : 2;
    const long long nb = (n + 256 * E - 1) / (256 * E);
    hipLaunchKernelGGL((lincomb_kernel<NQ, E>), dim3((unsigned)nb), dim3(256), 0, s, Y, ldy, nq, X, ldx, np, C, ldc, n,
                       alpha, beta);
}

template <int NQ>
void launch_dots_small(const double* X, long long ldx, int np, const double* Y, long long ldy, int nq, long long n,
                       long long chunk, long long nchunk, double* partial, hipStream_t s) {
    constexpr int PG = 64 / NQ;
    dim3 grid((unsigned)nchunk, (unsigned)((np + PG - 1) / PG));
    hipLaunchKernelGGL((dots_small_kernel<NQ, PG>), grid, dim3(256), 0, s, X, ldx, np, Y, ldy, nq, n, chunk, partial);
}
}  // namespace

size_t dots_partial_elems(int np, int nq, long long n) {
    return (size_t)(n / chunk_of(n) + 2) * np * nq;
}

void k_dots(const double* X, long long ldx, int np, const double* Y, long long ldy, int nq, long long n, double* G,
            int ldg, double* partial, hipStream_t s) {
    if (g_dry) return;
    if (np <= 0 || nq <= 0) return;
    // rows of the GEMM = the smaller set (skinny tiles when it is <= 16)
    const bool swapped = nq < np;
    const double* A = swapped ? Y : X;
    const double* B = swapped ? X : Y;
    const long long lda = swapped ? ldy : ldx, ldb = swapped ? ldx : ldy;
    const int M = swapped ? nq : np, N = swapped ? np : nq;
    const long long MN = (long long)M * N;
    // at most 64 products with one row group: the vector-ALU pass (A's rows against B's columns, the
    // partials laid out [chunk][M][N] as the GEMM's)
    if (n > 0 && M <= 16 && M * N <= 64 && (long long)N * ((M + 3) / 4 * 4) <= 64) {
        const long long ch = std::max<long long>(2048, (n + 511) / 512);
        const long long nch = (n + ch - 1) / ch;
        if (nch <= 65535 && nch * MN <= (long long)dots_partial_elems(np, nq, n)) {
            // rows of the output: the N operand rows against M (<= 16) operand rows
            if (M <= 1) launch_dots_small<1>(B, ldb, N, A, lda, M, n, ch, nch, partial, s);
            else if (M <= 2) launch_dots_small<2>(B, ldb, N, A, lda, M, n, ch, nch, partial, s);
            else if (M <= 4) launch_dots_small<4>(B, ldb, N, A, lda, M, n, ch, nch, partial, s);
            else if (M <= 8) launch_dots_small<8>(B, ldb, N, A, lda, M, n, ch, nch, partial, s);
            else launch_dots_small<16>(B, ldb, N, A, lda, M, n, ch, nch, partial, s);
            LAUNCHCHK();
            // partial[c][r][m] with r over the N operand: the transposed block of the GEMM's layout
            hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)MN), dim3(256), 0, s, partial, nch, N, M,
                               swapped ? 0 : 1, G, ldg);
            LAUNCHCHK();
            return;
        }
    }
    // up to 16 x 256 products: the fragment-streaming skinny kernel (partials [chunk][M][N] as the GEMM's)
    if (n > 0 && M <= 16 && N <= 256) {
        const long long nch = abt_skinny(M, N, n, A, lda, B, ldb, partial, (long long)dots_partial_elems(np, nq, n), s);
        if (nch > 0) {
            hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)MN), dim3(256), 0, s, partial, nch, M, N,
                               swapped ? 1 : 0, G, ldg);
            LAUNCHCHK();
            return;
        }
    }
    const long long CH = chunk_of(n);
    long long nchunk = (n + CH - 1) / CH;
    if (nchunk == 0) {
        k_fill(partial, MN, 0.0, s);
        nchunk = 1;
    } else {
        if (nchunk > 65535) fail(-1, "k_dots: vectors too long");
        Gemm g;
        g.M = M; g.N = N; g.K = (int)CH;
        g.Klast = (int)(n - (nchunk - 1) * CH);
        g.A = A; g.sAm = lda; g.sAk = 1; g.bA0 = CH;
        g.B = B; g.sBk = 1; g.sBn = ldb; g.bB0 = CH;
        g.C = partial; g.sCm = N; g.sCn = 1; g.bC0 = MN;
        g.nb0 = (int)nchunk;
        gemm(g, s);
    }
    hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)MN), dim3(256), 0, s, partial, nchunk, M, N,
                       swapped ? 1 : 0, G, ldg);
    LAUNCHCHK();
}

void k_lincomb(double* Y, long long ldy, int nq, const double* X, long long ldx, int np, const double* C, int ldc,
               long long n, double alpha, double beta, hipStream_t s) {
    if (g_dry) return;
    if (nq <= 0 || n <= 0) return;
    // few output rows: the streaming kernel (one pass over X, coefficients in scalar registers)
    if (nq <= 16 && np <= 128 && (n + 1023) / 1024 <= 0x7fffffffLL) {
        if (nq <= 1) launch_lincomb<1>(Y, ldy, nq, X, ldx, np, C, ldc, n, alpha, beta, s);
        else if (nq <= 2) launch_lincomb<2>(Y, ldy, nq, X, ldx, np, C, ldc, n, alpha, beta, s);
        else if (nq <= 4) launch_lincomb<4>(Y, ldy, nq, X, ldx, np, C, ldc, n, alpha, beta, s);
        else if (nq <= 8) launch_lincomb<8>(Y, ldy, nq, X, ldx, np, C, ldc, n, alpha, beta, s);
        else launch_lincomb<16>(Y, ldy, nq, X, ldx, np, C, ldc, n, alpha, beta, s);
        LAUNCHCHK();
        return;
    }
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
