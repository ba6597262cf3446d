// Symmetric eigensolvers in FP64: cyclic two-sided Jacobi with the round-robin
// ("circle method") ordering, so that every round rotates n/2 disjoint index pairs
// in parallel.  Order n <= 96 (the Rayleigh-Ritz subspace matrix): one workgroup, A and V in
// LDS.  Larger orders (the natural-orbital, recanonicalisation, exact-1p-block and
// natural-auxiliary-function matrices, one or a batch): the same ordering over blocks of 32
// rows, each round diagonalising the block pairs' sub-matrices in LDS and applying their
// orthogonal factors to A and V, two launches per round of block pairs.
#include "internal.h"
#include <algorithm>
#include <cmath>
#include <vector>

namespace adc3 {

namespace {

__device__ inline void pair_of(int r, int k, int np, int& p, int& q) {
    // players 0..np-1 (np even); player 0 fixed, others rotate by r
    auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + r) % (np - 1); };
    p = pos(k);
    q = pos(np - 1 - k);
    if (p > q) { int t = p; p = q; q = t; }
}

__device__ inline void rot_of(double app, double aqq, double apq, double& c, double& s) {
    if (apq == 0.0) { c = 1.0; s = 0.0; return; }
    double th = (aqq - app) / (2.0 * apq);
    double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
    c = 1.0 / sqrt(t * t + 1.0);
    s = t * c;
}

// ---------------- small: one workgroup, matrix and vectors in LDS ----------------
constexpr int SMALL_MAX = 96;
constexpr int SNT = 1024;

// Cyclic Jacobi on an n x n symmetric matrix held in LDS (row stride ld), one workgroup of SNT threads:
// sweeps of n - 1 (n even) rounds of n/2 disjoint rotations, until the off-diagonal squared norm is at most
// 1e-30 of the total (or max_sweeps).  V (same layout) accumulates the rotations on its columns.
__device__ void jacobi_lds(double* A, double* V, int n, int ld, int max_sweeps) {
    __shared__ double cs[SMALL_MAX / 2 + 1], sn[SMALL_MAX / 2 + 1];
    __shared__ int pp[SMALL_MAX / 2 + 1], qq[SMALL_MAX / 2 + 1];
    __shared__ double red[SNT / 64];
    __shared__ double red2[SNT / 64];
    const int tid = threadIdx.x;
    const int np = n + (n & 1);
    const int npair = np / 2;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int t = tid; t < n * n; t += SNT) {
            int i = t / n, j = t % n;
            double a = A[i * ld + j];
            tot += a * a;
            if (i != j) off += a * a;
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_down(off, o, 64);
            tot += __shfl_down(tot, o, 64);
        }
        if ((tid & 63) == 0) { red[tid >> 6] = off; red2[tid >> 6] = tot; }
        __syncthreads();
        double offs = 0.0, tots = 0.0;
        for (int k = 0; k < SNT / 64; ++k) { offs += red[k]; tots += red2[k]; }
        __syncthreads();
        if (offs <= 1e-30 * tots || offs == 0.0) break;
        for (int r = 0; r < np - 1; ++r) {
            if (tid < npair) {
                int p, q;
                pair_of(r, tid, np, p, q);
                double c = 1.0, s = 0.0;
                if (q < n) rot_of(A[p * ld + p], A[q * ld + q], A[p * ld + q], c, s);
                pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
            }
            __syncthreads();
            // The round's rotations act on disjoint index pairs, so each 2x2 block (row pair k1, column
            // pair k2) of A is updated in place by one thread: rows rotated first, then columns, the same
            // arithmetic as a full row pass followed by a full column pass.  A pair whose q is past n
            // (odd n) is the single index p with the identity rotation.  V's columns are rotated alongside.
            for (int t = tid; t < npair * npair; t += SNT) {
                const int k1 = t / npair, k2 = t - (t / npair) * npair;
                const int p1 = pp[k1], q1 = qq[k1], p2 = pp[k2], q2 = qq[k2];
                const bool h1 = q1 < n, h2 = q2 < n;
                const double c1 = cs[k1], s1 = sn[k1], c2 = cs[k2], s2 = sn[k2];
                const double x00 = A[p1 * ld + p2];
                const double x01 = h2 ? A[p1 * ld + q2] : 0.0;
                const double x10 = h1 ? A[q1 * ld + p2] : 0.0;
                const double x11 = h1 && h2 ? A[q1 * ld + q2] : 0.0;
                // rows
                double y00 = x00, y01 = x01, y10 = x10, y11 = x11;
                if (h1) {
                    y00 = c1 * x00 - s1 * x10;
                    y10 = s1 * x00 + c1 * x10;
                    y01 = c1 * x01 - s1 * x11;
                    y11 = s1 * x01 + c1 * x11;
                }
                // columns
                if (h2) {
                    A[p1 * ld + p2] = c2 * y00 - s2 * y01;
                    A[p1 * ld + q2] = s2 * y00 + c2 * y01;
                    if (h1) {
                        A[q1 * ld + p2] = c2 * y10 - s2 * y11;
                        A[q1 * ld + q2] = s2 * y10 + c2 * y11;
                    }
                } else {
                    A[p1 * ld + p2] = y00;
                    if (h1) A[q1 * ld + p2] = y10;
                }
            }
            for (int t = tid; t < npair * n; t += SNT) {
                int k = t / n, i = t % n;
                int p = pp[k], q = qq[k];
                if (q >= n) continue;
                double c = cs[k], s = sn[k];
                double vip = V[i * ld + p], viq = V[i * ld + q];
                V[i * ld + p] = c * vip - s * viq;
                V[i * ld + q] = s * vip + c * viq;
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(SNT) void jacobi_small_kernel(double* Ag, int n, double* w, double* Vg) {
    extern __shared__ double sm[];
    const int ld = n + 1;
    double* A = sm;
    double* V = sm + (size_t)n * ld;
    const int tid = threadIdx.x;
    for (int t = tid; t < n * n; t += SNT) {
        int i = t / n, j = t % n;
        A[i * ld + j] = Ag[t];
        V[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_lds(A, V, n, ld, 60);
    for (int t = tid; t < n * n; t += SNT) {
        int i = t / n, j = t % n;
        Vg[t] = V[i * ld + j];
    }
    for (int i = tid; i < n; i += SNT) w[i] = A[i * ld + i];
}

// Per matrix of the batch (one workgroup each): off-diagonal and total squared norms into nrm[2b..2b+1];
// an active matrix whose off-diagonal norm has reached the threshold (or is not finite) is marked done.
__global__ void offnorm_batched_kernel(const double* A, int n, double* nrm, int* active) {
    const int bm = blockIdx.x;
    if (!active[bm]) return;
    const double* Ab = A + (long long)bm * n * n;
    __shared__ double r1[16], r2[16];
    double off = 0.0, tot = 0.0;
    long long nn = (long long)n * n;
    for (long long t = threadIdx.x; t < nn; t += blockDim.x) {
        double a = Ab[t];
        tot += a * a;
        if (t / n != t % n) off += a * a;
    }
    for (int o = 32; o > 0; o >>= 1) {
        off += __shfl_down(off, o, 64);
        tot += __shfl_down(tot, o, 64);
    }
    if ((threadIdx.x & 63) == 0) { r1[threadIdx.x >> 6] = off; r2[threadIdx.x >> 6] = tot; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { a += r1[k]; b += r2[k]; }
        nrm[2 * bm] = a;
        nrm[2 * bm + 1] = b;
        if (!(a == a && b == b) || !(b < INFINITY) || a <= 1e-30 * b || a == 0.0) active[bm] = 0;
    }
}

// w[b][i] = A_b[i][i], A_b taken from A or A2 as src[b] says
__global__ void diag_out_batched_kernel(const double* A, const double* A2, const int* src, int n, double* w) {
    const int bm = blockIdx.y, i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* Ab = (src[bm] ? A2 : A) + (long long)bm * n * n;
    w[(long long)bm * n + i] = Ab[(long long)i * n + i];
}

__global__ void eye_kernel(double* V, int n) {
    long long nn = (long long)n * n;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nn; t += (long long)gridDim.x * blockDim.x)
        V[t] = (t / n == t % n) ? 1.0 : 0.0;
}

// ascending (desc=0) or descending (desc=1) order; ties by index; sign: largest |.| of
// each column positive (first index on ties)
__global__ void sort_eig_kernel(double* w, double* V, int n, int desc, double* wtmp, double* Vtmp) {
    // rank
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double wi = w[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            double wj = w[j];
            bool before = desc ? (wj > wi || (wj == wi && j < i)) : (wj < wi || (wj == wi && j < i));
            rank += before;
        }
        wtmp[rank] = wi;
        // copy column i to column rank with sign fix
        double best = -1.0, sgn = 1.0;
        for (int r = 0; r < n; ++r) {
            double x = V[(long long)r * n + i];
            if (fabs(x) > best) { best = fabs(x); sgn = x < 0 ? -1.0 : 1.0; }
        }
        for (int r = 0; r < n; ++r) Vtmp[(long long)r * n + rank] = sgn * V[(long long)r * n + i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = wtmp[i];
    for (long long t = threadIdx.x; t < (long long)n * n; t += blockDim.x) V[t] = Vtmp[t];
}

// ---------------- large: block Jacobi, two launches per round of block pairs ----------------
// The matrix is cut into blocks of BJ rows (the last one shorter).  Every round pairs the blocks in the
// same round-robin order as the scalar rounds (with a bye when their count is odd); bj_solve_kernel
// diagonalises, for each pair, the symmetric sub-matrix on the pair's rows and columns (at most BSUB)
// in LDS with the one-workgroup Jacobi, and writes its orthogonal factor Q_k; bj_apply_kernel then applies
// every pair's factor at once, A <- P^T A P and V <- V P with P block-diagonal over the pairs' index sets,
// each tile (pair p's rows, pair q's columns) of A, and each BSUB-row slab of V's pair-q columns, by one
// workgroup.  Every element of A lies in exactly one tile, so A is updated in place.
constexpr int BJ = 32, BSUB = 2 * BJ, BL = BSUB + 1;
// Jacobi sweeps per sub-problem and round: the outer sweeps converge the whole matrix either way, and two
// inner sweeps measured fastest (1, 2 and full inner convergence compared at n = 200 and 600, random and
// density-like spectra, and in the SS-FNO solve)
constexpr int BJ_INNER = 2;

// the pair k of round r: first block's first row b0 and size m0, second block's b1 and m1 (m1 = 0 for the bye)
__device__ inline void bj_pair(int r, int k, int npb, int nblk, int n, int& b0, int& m0, int& b1, int& m1) {
    int I, J;
    pair_of(r, k, npb, I, J);
    b0 = I * BJ;
    m0 = min(BJ, n - b0);
    if (J < nblk) {
        b1 = J * BJ;
        m1 = min(BJ, n - b1);
    } else {
        b1 = 0;
        m1 = 0;
    }
}
__device__ inline int bj_row(int t, int b0, int m0, int b1) { return t < m0 ? b0 + t : b1 + (t - m0); }

// grid (npb / 2, batch); Q [batch][npb / 2][BSUB][BSUB]
__global__ __launch_bounds__(SNT) void bj_solve_kernel(const double* A, double* Q, int n, int nblk, int npb, int r,
                                                       int sweeps, const int* active) {
    const int bm = blockIdx.y;
    if (active && !active[bm]) return;
    const double* Ab = A + (long long)bm * n * n;
    double* Qb = Q + ((long long)bm * (npb / 2) + blockIdx.x) * BSUB * BSUB;
    int b0, m0, b1, m1;
    bj_pair(r, blockIdx.x, npb, nblk, n, b0, m0, b1, m1);
    const int ms = m0 + m1, ld = ms + 1;
    extern __shared__ double sm[];
    double* As = sm;
    double* Vs = sm + (size_t)ms * ld;
    for (int t = threadIdx.x; t < ms * ms; t += SNT) {
        const int i = t / ms, j = t - (t / ms) * ms;
        const long long gi = bj_row(i, b0, m0, b1), gj = bj_row(j, b0, m0, b1);
        As[i * ld + j] = 0.5 * (Ab[gi * n + gj] + Ab[gj * n + gi]);
        Vs[i * ld + j] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_lds(As, Vs, ms, ld, sweeps);
    // one Newton-Schulz step, Q = V (3 I - V^T V) / 2, takes the factor's departure from orthogonality (the
    // rounding of its many rotations) from e to about e^2, so that it does not add up over the rounds
    // applied to the eigenvectors; G = V^T V goes where the sub-matrix was
    double* G = As;
    for (int t = threadIdx.x; t < ms * ms; t += SNT) {
        const int i = t / ms, j = t - (t / ms) * ms;
        double acc = 0.0;
        for (int k = 0; k < ms; ++k) acc += Vs[k * ld + i] * Vs[k * ld + j];
        G[i * ld + j] = acc;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ms * ms; t += SNT) {
        const int i = t / ms, j = t - (t / ms) * ms;
        double acc = 0.0;
        for (int k = 0; k < ms; ++k) acc += Vs[i * ld + k] * G[k * ld + j];
        Qb[i * BSUB + j] = 1.5 * Vs[i * ld + j] - 0.5 * acc;
    }
}

// grid (npb / 2, npb / 2 + ceil(n / BSUB), batch): y < npb / 2 the A tile (pair y's rows, pair x's columns),
// otherwise the V slab of rows BSUB (y - npb / 2) .. on pair x's columns
__global__ __launch_bounds__(256) void bj_apply_kernel(double* A, double* V, const double* Q, int n, int nblk, int npb,
                                                       int r, const int* active) {
    const int bm = blockIdx.z;
    if (active && !active[bm]) return;
    const int npair = npb / 2;
    const long long nn = (long long)n * n;
    double* Ab = A + bm * nn;
    double* Vb = V + bm * nn;
    const double* Qb = Q + (long long)bm * npair * BSUB * BSUB;
    extern __shared__ double sm[];
    double* Qc = sm;               // column pair's factor [mc][BL]
    double* X = sm + BSUB * BL;    // the tile or slab [rows][BL]
    double* T = sm + 2 * BSUB * BL;
    double* Qr = sm + 3 * BSUB * BL;
    int c0, cm0, c1, cm1;
    bj_pair(r, blockIdx.x, npb, nblk, n, c0, cm0, c1, cm1);
    const int mc = cm0 + cm1;
    const double* Qcg = Qb + (long long)blockIdx.x * BSUB * BSUB;
    for (int t = threadIdx.x; t < mc * mc; t += 256) {
        const int i = t / mc, j = t - (t / mc) * mc;
        Qc[i * BL + j] = Qcg[i * BSUB + j];
    }
    if ((int)blockIdx.y < npair) {
        int r0, rm0, r1, rm1;
        bj_pair(r, blockIdx.y, npb, nblk, n, r0, rm0, r1, rm1);
        const int mr = rm0 + rm1;
        const double* Qrg = Qb + (long long)blockIdx.y * BSUB * BSUB;
        for (int t = threadIdx.x; t < mr * mr; t += 256) {
            const int i = t / mr, j = t - (t / mr) * mr;
            Qr[i * BL + j] = Qrg[i * BSUB + j];
        }
        for (int t = threadIdx.x; t < mr * mc; t += 256) {
            const int i = t / mc, j = t - (t / mc) * mc;
            X[i * BL + j] = Ab[(long long)bj_row(i, r0, rm0, r1) * n + bj_row(j, c0, cm0, c1)];
        }
        __syncthreads();
        // T = Qr^T X
        for (int t = threadIdx.x; t < mr * mc; t += 256) {
            const int i = t / mc, j = t - (t / mc) * mc;
            double acc = 0.0;
            for (int k = 0; k < mr; ++k) acc += Qr[k * BL + i] * X[k * BL + j];
            T[i * BL + j] = acc;
        }
        __syncthreads();
        // A tile = T Qc
        for (int t = threadIdx.x; t < mr * mc; t += 256) {
            const int i = t / mc, j = t - (t / mc) * mc;
            double acc = 0.0;
            for (int k = 0; k < mc; ++k) acc += T[i * BL + k] * Qc[k * BL + j];
            Ab[(long long)bj_row(i, r0, rm0, r1) * n + bj_row(j, c0, cm0, c1)] = acc;
        }
    } else {
        const int row0 = ((int)blockIdx.y - npair) * BSUB;
        const int mr = min(BSUB, n - row0);
        for (int t = threadIdx.x; t < mr * mc; t += 256) {
            const int i = t / mc, j = t - (t / mc) * mc;
            X[i * BL + j] = Vb[(long long)(row0 + i) * n + bj_row(j, c0, cm0, c1)];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < mr * mc; t += 256) {
            const int i = t / mc, j = t - (t / mc) * mc;
            double acc = 0.0;
            for (int k = 0; k < mc; ++k) acc += X[i * BL + k] * Qc[k * BL + j];
            Vb[(long long)(row0 + i) * n + bj_row(j, c0, cm0, c1)] = acc;
        }
    }
}
}  // namespace

void eig_small(double* A, int n, double* w, double* V, hipStream_t s) {
    if (g_dry) return;
    if (n <= 0) return;
    if (n > SMALL_MAX) fail(-1, "eig_small: n too large");
    size_t lds = 2 * (size_t)n * (n + 1) * sizeof(double);
    // once per process (thread-safe initialisation; retried if it throws)
    static const bool attr_set = [] {
        HIPCHK(hipFuncSetAttribute((const void*)jacobi_small_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(2 * SMALL_MAX * (SMALL_MAX + 1) * sizeof(double))));
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL(jacobi_small_kernel, dim3(1), dim3(SNT), lds, s, A, n, w, V);
    LAUNCHCHK();
}


namespace {
// doubles of scratch the block solver takes for nb matrices of order n: the pairs' factors, norms, flags
size_t block_scratch(int n, int nb) {
    const long long nblk = (n + BJ - 1) / BJ, npair = (nblk + (nblk & 1)) / 2;
    return (size_t)nb * npair * BSUB * BSUB + 4 * (size_t)nb + 8;
}

// nb symmetric matrices of order n > SMALL_MAX, [nb][n][n]: eigenvalues w [nb][n] (unsorted) and
// eigenvectors V [nb][n][n] (columns), A overwritten; each matrix stops at its own convergence.
void eig_block(double* A, int n, int nb, double* w, double* V, double* scratch, hipStream_t s) {
    static const bool attr_set = [] {
        HIPCHK(hipFuncSetAttribute((const void*)bj_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(2 * BSUB * BL * sizeof(double))));
        HIPCHK(hipFuncSetAttribute((const void*)bj_apply_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(4 * BSUB * BL * sizeof(double))));
        return true;
    }();
    (void)attr_set;
    const long long nn = (long long)n * n;
    const int nblk = (n + BJ - 1) / BJ, npb = nblk + (nblk & 1), npair = npb / 2;
    double* Q = scratch;
    double* nrm = Q + (long long)nb * npair * BSUB * BSUB;  // [nb][2]
    int* active = (int*)(nrm + 2 * (long long)nb);           // [nb]
    int* src = active + nb;                                  // [nb], zeros: the matrices stay in A
    std::vector<int> hact(nb, 1), hzero(nb, 0);
    std::vector<double> hn(2 * (size_t)nb);
    HIPCHK(hipMemcpyAsync(active, hact.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(src, hzero.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    for (int b = 0; b < nb; ++b) {
        hipLaunchKernelGGL(eye_kernel, dim3(256), dim3(256), 0, s, V + b * nn, n);
        LAUNCHCHK();
    }
    const dim3 gs(npair, nb), ga(npair, npair + (n + BSUB - 1) / BSUB, nb);
    const size_t lds_s = 2 * (size_t)BSUB * BL * sizeof(double), lds_a = 4 * (size_t)BSUB * BL * sizeof(double);
    for (int sweep = 0; sweep < 60; ++sweep) {
        hipLaunchKernelGGL(offnorm_batched_kernel, dim3(nb), dim3(1024), 0, s, A, n, nrm, active);
        LAUNCHCHK();
        std::vector<int> now(nb);
        HIPCHK(hipMemcpyAsync(now.data(), active, nb * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hn.data(), nrm, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int left = 0;
        for (int b = 0; b < nb; ++b) {
            if (hact[b] && !now[b] && (!std::isfinite(hn[2 * b]) || !std::isfinite(hn[2 * b + 1])))
                fail(-4, "eigensolver: non-finite matrix");
            hact[b] = now[b];
            left += now[b];
        }
        if (left == 0) break;
        for (int r = 0; r < npb - 1; ++r) {
            hipLaunchKernelGGL(bj_solve_kernel, gs, dim3(SNT), lds_s, s, A, Q, n, nblk, npb, r, BJ_INNER, active);
            hipLaunchKernelGGL(bj_apply_kernel, ga, dim3(256), lds_a, s, A, V, Q, n, nblk, npb, r, active);
        }
        LAUNCHCHK();
    }
    hipLaunchKernelGGL(diag_out_batched_kernel, dim3((n + 255) / 256, nb), dim3(256), 0, s, A, A, src, n, w);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));  // the host arrays of the copies above go out of scope here
}
}  // namespace

// the block solver's factors, norms and flags
size_t eig_large_scratch(int n) { return std::max((size_t)n * n + 8, block_scratch(n, 1)); }

void eig_large(double* A, int n, double* w, double* V, double* scratch, hipStream_t s) {
    if (g_dry) return;
    ProfScope prof(PROF_EIG, s, 0.0, 0.0);
    if (n <= 0) return;
    if (n <= SMALL_MAX) { eig_small(A, n, w, V, s); return; }
    eig_block(A, n, 1, w, V, scratch, s);
}

// the block solver's factors, norms and flags of the nb matrices
size_t eig_batched_scratch(int n, int nb) { return std::max((size_t)nb * n * n + 4 * (size_t)nb + 8, block_scratch(n, nb)); }

void eig_batched(double* A, int n, int nb, double* w, double* V, double* scratch, hipStream_t s) {
    if (g_dry) return;
    ProfScope prof(PROF_EIG, s, 0.0, 0.0);
    if (n <= 0 || nb <= 0) return;
    const long long nn = (long long)n * n;
    if (n <= SMALL_MAX) {
        for (int b = 0; b < nb; ++b) eig_small(A + b * nn, n, w + (long long)b * n, V + b * nn, s);
        return;
    }
    eig_block(A, n, nb, w, V, scratch, s);
}

void k_sort_eig(double* w, double* V, int n, int desc, double* wtmp, double* Vtmp, hipStream_t s) {
    if (g_dry) return;
    if (n <= 0) return;
    hipLaunchKernelGGL(sort_eig_kernel, dim3(1), dim3(1024), 0, s, w, V, n, desc, wtmp, Vtmp);
    LAUNCHCHK();
}

}  // namespace adc3
