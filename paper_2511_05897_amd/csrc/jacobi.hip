// Symmetric eigensolvers in FP64: cyclic two-sided Jacobi with the round-robin
// ("circle method") ordering, so that every round rotates n/2 disjoint index pairs
// in parallel.  Used for the Rayleigh-Ritz subspace matrix (small, one workgroup,
// LDS resident), the natural-orbital and recanonicalisation matrices and the
// natural-auxiliary-function matrix (large, one launch per round, two buffers of A).
#include "internal.h"
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

__global__ __launch_bounds__(SNT) void jacobi_small_kernel(double* Ag, int n, double* w, double* Vg) {
    extern __shared__ double sm[];
    const int ld = n + 1;
    double* A = sm;
    double* V = sm + (size_t)n * ld;
    __shared__ double cs[SMALL_MAX / 2 + 1], sn[SMALL_MAX / 2 + 1];
    __shared__ int pp[SMALL_MAX / 2 + 1], qq[SMALL_MAX / 2 + 1];
    __shared__ double red[SNT / 64];
    __shared__ double red2[SNT / 64];
    const int tid = threadIdx.x;
    for (int t = tid; t < n * n; t += SNT) {
        int i = t / n, j = t % n;
        A[i * ld + j] = Ag[t];
        V[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int np = n + (n & 1);
    const int npair = np / 2;
    for (int sweep = 0; sweep < 60; ++sweep) {
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
    for (int t = tid; t < n * n; t += SNT) {
        int i = t / n, j = t % n;
        Vg[t] = V[i * ld + j];
    }
    for (int i = tid; i < n; i += SNT) w[i] = A[i * ld + i];
}

// ---------------- large: global memory, one launch per round ----------------
// One round in one launch: every workgroup forms all the round's rotations from Ain (which no
// workgroup writes in this round) in LDS, then applies its share of the block updates into Aout.
// Every element of A belongs to exactly one (row pair, column pair) block, so Aout is written in full;
// V is updated in place (each (row, pair) element by one thread).
__global__ void jacobi_round_kernel(const double* Ain, double* Aout, double* V, int n, int np, int r) {
    extern __shared__ double csh[];  // [2 * npair]
    const int npair = np / 2;
    for (int k = threadIdx.x; k < npair; k += blockDim.x) {
        int p, q;
        pair_of(r, k, np, p, q);
        double c = 1.0, s = 0.0;
        if (q < n) rot_of(Ain[(long long)p * n + p], Ain[(long long)q * n + q], Ain[(long long)p * n + q], c, s);
        csh[2 * k] = c;
        csh[2 * k + 1] = s;
    }
    __syncthreads();
    long long nblk = (long long)npair * npair;
    long long nv = (long long)n * npair;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nblk + nv;
         t += (long long)gridDim.x * blockDim.x) {
        if (t < nblk) {
            int k1 = (int)(t / npair), k2 = (int)(t % npair);
            int p1, q1, p2, q2;
            pair_of(r, k1, np, p1, q1);
            pair_of(r, k2, np, p2, q2);
            double c1 = csh[2 * k1], s1 = csh[2 * k1 + 1], c2 = csh[2 * k2], s2 = csh[2 * k2 + 1];
            bool v1 = q1 < n, v2 = q2 < n;
            double a = Ain[(long long)p1 * n + p2];
            double b = v2 ? Ain[(long long)p1 * n + q2] : 0.0;
            double c = v1 ? Ain[(long long)q1 * n + p2] : 0.0;
            double d = (v1 && v2) ? Ain[(long long)q1 * n + q2] : 0.0;
            double ra = c1 * a - s1 * c, rb = c1 * b - s1 * d;
            double rc = s1 * a + c1 * c, rd = s1 * b + c1 * d;
            double na = c2 * ra - s2 * rb, nb = s2 * ra + c2 * rb;
            double nc = c2 * rc - s2 * rd, nd = s2 * rc + c2 * rd;
            Aout[(long long)p1 * n + p2] = na;
            if (v2) Aout[(long long)p1 * n + q2] = nb;
            if (v1) Aout[(long long)q1 * n + p2] = nc;
            if (v1 && v2) Aout[(long long)q1 * n + q2] = nd;
        } else {
            long long u = t - nblk;
            int k = (int)(u / n), i = (int)(u % n);
            int p, q;
            pair_of(r, k, np, p, q);
            if (q >= n) continue;
            double c = csh[2 * k], s = csh[2 * k + 1];
            double vip = V[(long long)i * n + p], viq = V[(long long)i * n + q];
            V[(long long)i * n + p] = c * vip - s * viq;
            V[(long long)i * n + q] = s * vip + c * viq;
        }
    }
}

// Batched round: blockIdx.y picks the matrix (order n, contiguous [nb][n][n] buffers); matrices whose
// flag is 0 (converged) are left as they are.
__global__ void jacobi_round_batched_kernel(const double* Ain, double* Aout, double* Vb, int n, int np, int r,
                                            const int* active) {
    const int bm = blockIdx.y;
    if (!active[bm]) return;
    const long long nn = (long long)n * n;
    const double* Ai = Ain + bm * nn;
    double* Ao = Aout + bm * nn;
    double* V = Vb + bm * nn;
    extern __shared__ double csh[];  // [2 * npair]
    const int npair = np / 2;
    for (int k = threadIdx.x; k < npair; k += blockDim.x) {
        int p, q;
        pair_of(r, k, np, p, q);
        double c = 1.0, s = 0.0;
        if (q < n) rot_of(Ai[(long long)p * n + p], Ai[(long long)q * n + q], Ai[(long long)p * n + q], c, s);
        csh[2 * k] = c;
        csh[2 * k + 1] = s;
    }
    __syncthreads();
    long long nblk = (long long)npair * npair;
    long long nv = (long long)n * npair;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nblk + nv;
         t += (long long)gridDim.x * blockDim.x) {
        if (t < nblk) {
            int k1 = (int)(t / npair), k2 = (int)(t % npair);
            int p1, q1, p2, q2;
            pair_of(r, k1, np, p1, q1);
            pair_of(r, k2, np, p2, q2);
            double c1 = csh[2 * k1], s1 = csh[2 * k1 + 1], c2 = csh[2 * k2], s2 = csh[2 * k2 + 1];
            bool v1 = q1 < n, v2 = q2 < n;
            double a = Ai[(long long)p1 * n + p2];
            double b = v2 ? Ai[(long long)p1 * n + q2] : 0.0;
            double c = v1 ? Ai[(long long)q1 * n + p2] : 0.0;
            double d = (v1 && v2) ? Ai[(long long)q1 * n + q2] : 0.0;
            double ra = c1 * a - s1 * c, rb = c1 * b - s1 * d;
            double rc = s1 * a + c1 * c, rd = s1 * b + c1 * d;
            double na = c2 * ra - s2 * rb, nb = s2 * ra + c2 * rb;
            double nc = c2 * rc - s2 * rd, nd = s2 * rc + c2 * rd;
            Ao[(long long)p1 * n + p2] = na;
            if (v2) Ao[(long long)p1 * n + q2] = nb;
            if (v1) Ao[(long long)q1 * n + p2] = nc;
            if (v1 && v2) Ao[(long long)q1 * n + q2] = nd;
        } else {
            long long u = t - nblk;
            int k = (int)(u / n), i = (int)(u % n);
            int p, q;
            pair_of(r, k, np, p, q);
            if (q >= n) continue;
            double c = csh[2 * k], s = csh[2 * k + 1];
            double vip = V[(long long)i * n + p], viq = V[(long long)i * n + q];
            V[(long long)i * n + p] = c * vip - s * viq;
            V[(long long)i * n + q] = s * vip + c * viq;
        }
    }
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

__global__ void offnorm_kernel(const double* A, int n, double* out) {
    __shared__ double r1[16], r2[16];
    double off = 0.0, tot = 0.0;
    long long nn = (long long)n * n;
    for (long long t = threadIdx.x; t < nn; t += blockDim.x) {
        double a = A[t];
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
        out[0] = a;
        out[1] = b;
    }
}

__global__ void eye_kernel(double* V, int n) {
    long long nn = (long long)n * n;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nn; t += (long long)gridDim.x * blockDim.x)
        V[t] = (t / n == t % n) ? 1.0 : 0.0;
}

__global__ void diag_out_kernel(const double* A, int n, double* w) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = A[(long long)i * n + i];
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

// second copy of A (rounds alternate between the two) + norms
size_t eig_large_scratch(int n) { return (size_t)n * n + 8; }

void eig_large(double* A, int n, double* w, double* V, double* scratch, hipStream_t s) {
    if (g_dry) return;
    ProfScope prof(PROF_EIG, s, 0.0, 0.0);
    if (n <= 0) return;
    if (n <= SMALL_MAX) { eig_small(A, n, w, V, s); return; }
    const int np = n + (n & 1);
    double* A2 = scratch;                  // n*n doubles: the other buffer of the rounds
    double* nrm = scratch + (long long)n * n;  // 2 doubles
    hipLaunchKernelGGL(eye_kernel, dim3(256), dim3(256), 0, s, V, n);
    LAUNCHCHK();
    long long work = (long long)(np / 2) * (np / 2) + (long long)n * (np / 2);
    unsigned gb = (unsigned)std::min<long long>((work + 255) / 256, 4096);
    const size_t lds = (size_t)np * sizeof(double);  // 2 * (np/2) rotation coefficients
    if (lds > 64 * 1024) fail(-1, "eig_large: n too large");
    double* cur = A;
    double* nxt = A2;
    double hn[2];
    for (int sweep = 0; sweep < 60; ++sweep) {
        hipLaunchKernelGGL(offnorm_kernel, dim3(1), dim3(1024), 0, s, cur, n, nrm);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(hn, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!std::isfinite(hn[0]) || !std::isfinite(hn[1])) fail(-4, "eigensolver: non-finite matrix");
        if (hn[0] <= 1e-30 * hn[1] || hn[0] == 0.0) break;
        for (int r = 0; r < np - 1; ++r) {
            hipLaunchKernelGGL(jacobi_round_kernel, dim3(gb), dim3(256), lds, s, cur, nxt, V, n, np, r);
            std::swap(cur, nxt);
        }
        LAUNCHCHK();
    }
    hipLaunchKernelGGL(diag_out_kernel, dim3((n + 255) / 256), dim3(256), 0, s, cur, n, w);
    LAUNCHCHK();
}

// second copies of the nb matrices, norms, flags
size_t eig_batched_scratch(int n, int nb) { return (size_t)nb * n * n + 4 * (size_t)nb + 8; }

void eig_batched(double* A, int n, int nb, double* w, double* V, double* scratch, hipStream_t s) {
    if (g_dry) return;
    ProfScope prof(PROF_EIG, s, 0.0, 0.0);
    if (n <= 0 || nb <= 0) return;
    const long long nn = (long long)n * n;
    if (n <= SMALL_MAX || nb == 1) {
        for (int b = 0; b < nb; ++b) eig_large(A + b * nn, n, w + (long long)b * n, V + b * nn, scratch, s);
        return;
    }
    const int np = n + (n & 1);
    double* A2 = scratch;
    double* nrm = scratch + nb * nn;                 // [nb][2]
    int* active = (int*)(nrm + 2 * (long long)nb);   // [nb]
    int* src = active + nb;                           // [nb]
    std::vector<int> hact(nb, 1), hsrc(nb, 0);
    std::vector<double> hn(2 * (size_t)nb);
    HIPCHK(hipMemcpyAsync(active, hact.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    for (int b = 0; b < nb; ++b) {
        hipLaunchKernelGGL(eye_kernel, dim3(256), dim3(256), 0, s, V + b * nn, n);
        LAUNCHCHK();
    }
    long long work = (long long)(np / 2) * (np / 2) + (long long)n * (np / 2);
    unsigned gb = (unsigned)std::min<long long>((work + 255) / 256, 4096);
    const size_t lds = (size_t)np * sizeof(double);
    if (lds > 64 * 1024) fail(-1, "eig_batched: n too large");
    int parity = 0;  // 0: current matrices in A, 1: in A2
    for (int sweep = 0; sweep < 60; ++sweep) {
        hipLaunchKernelGGL(offnorm_batched_kernel, dim3(nb), dim3(1024), 0, s, parity ? A2 : A, n, nrm, active);
        LAUNCHCHK();
        std::vector<int> now(nb);
        HIPCHK(hipMemcpyAsync(now.data(), active, nb * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hn.data(), nrm, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int left = 0;
        for (int b = 0; b < nb; ++b) {
            if (hact[b] && !now[b]) {
                if (!std::isfinite(hn[2 * b]) || !std::isfinite(hn[2 * b + 1]))
                    fail(-4, "eigensolver: non-finite matrix");
                hsrc[b] = parity;  // converged here: its matrix stays in the current buffer
            }
            hact[b] = now[b];
            left += now[b];
        }
        if (left == 0) break;
        for (int r = 0; r < np - 1; ++r) {
            hipLaunchKernelGGL(jacobi_round_batched_kernel, dim3(gb, nb), dim3(256), lds, s, parity ? A2 : A,
                               parity ? A : A2, V, n, np, r, active);
            parity ^= 1;
        }
        LAUNCHCHK();
    }
    for (int b = 0; b < nb; ++b)
        if (hact[b]) hsrc[b] = parity;  // not converged within the sweep limit: the last buffer
    HIPCHK(hipMemcpyAsync(src, hsrc.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(diag_out_batched_kernel, dim3((n + 255) / 256, nb), dim3(256), 0, s, A, A2, src, n, w);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));  // the host arrays of the copies above go out of scope here
}

void k_sort_eig(double* w, double* V, int n, int desc, double* wtmp, double* Vtmp, hipStream_t s) {
    if (g_dry) return;
    if (n <= 0) return;
    hipLaunchKernelGGL(sort_eig_kernel, dim3(1), dim3(1024), 0, s, w, V, n, desc, wtmp, Vtmp);
    LAUNCHCHK();
}

}  // namespace adc3
